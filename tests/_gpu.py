"""GPU-side test helpers: upload graphs, run walks through the C ABI, compare with the
oracle.  Only the tests import this module."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_2512_00705_amd as fw

MARGIN = 1e-6  # a float decision within this relative gap is a flagged boundary


class GpuGraph:
    def __init__(self, g: dict, on_device: bool = True, preprocess: bool = True, index: bool = False,
                 alias: bool = False, label_alias: bool = False):
        self.g = g
        self.nv, self.ne = int(g["nv"]), int(g["ne"])
        dev = torch.device("cuda:0")
        keys = ("row_ptr", "col", "h", "label", "h8")  # h8: 8-bit weight codes with g["h_scale"]
        if on_device:
            self.t = {k: torch.from_numpy(np.ascontiguousarray(g[k])).to(dev) for k in keys if g.get(k) is not None}
            arrs = {k: self.t.get(k) for k in keys}
        else:
            arrs = {k: (None if g.get(k) is None else np.ascontiguousarray(g[k])) for k in keys}
            self.host = arrs
        self.handle = fw.fw_graph_create(self.nv, self.ne, arrs["row_ptr"], arrs["col"], arrs["h"], arrs["label"],
                                         on_device=on_device, h8=arrs["h8"], h_scale=float(g.get("h_scale", 0.0)))
        if preprocess:
            fw.fw_graph_preprocess(self.handle)
        if index:
            fw.fw_graph_build_index(self.handle)
        if alias:
            fw.fw_graph_build_alias(self.handle)
        if label_alias:
            fw.fw_graph_build_label_alias(self.handle)
        torch.cuda.synchronize()

    def close(self):
        if self.handle:
            torch.cuda.synchronize()
            fw.fw_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fw_logic(lg: oracle.Logic):
    if lg.kind == oracle.NODE2VEC:
        return fw.fw_logic_node2vec(lg.p, lg.q, lg.weighted)
    if lg.kind == oracle.SECOND_PR:
        return fw.fw_logic_second_pr(lg.gamma, lg.weighted)
    return fw.fw_logic_metapath(list(lg.schema), lg.weighted)


def fw_plan(pl: oracle.Plan, **speed):
    assert pl.lanes == 64 and pl.jump and pl.bound_scale == 1.0
    return fw.fw_plan_default(rho=pl.rho, d_lo=pl.d_lo, rjs_cap=pl.rjs_cap, bound=pl.bound, proposal=pl.proposal,
                              hub_deg=pl.hub_deg, hub_lanes=pl.hub_lanes, rvs_share=int(pl.rvs_share), **speed)


def gpu_walk(gg: GpuGraph, lg: oracle.Logic, pl: oracle.Plan, strategy: int, starts: np.ndarray, L: int,
             seed: int, counters: bool = True, **speed):
    """counters=False launches without the device counter array, as the benchmark's timed
    launches run (the library then runs its counter-free kernel variant); stats is {}."""
    dev = torch.device("cuda:0")
    n = int(starts.shape[0])
    st = torch.from_numpy(np.ascontiguousarray(starts, np.int32)).to(dev)
    paths = torch.full((max(n, 1), L + 1), -7, dtype=torch.int32, device=dev)
    lengths = torch.full((max(n, 1),), -7, dtype=torch.int32, device=dev)
    stats = torch.zeros(fw.FW_NSTATS, dtype=torch.int64, device=dev) if counters else None
    fw.fw_walk(gg.handle, fw_logic(lg), fw_plan(pl, **speed), strategy, st, n, L, seed, paths, lengths, stats)
    torch.cuda.synchronize()
    return (paths[:n].cpu().numpy(), lengths[:n].cpu().numpy(),
            dict(zip(fw.STAT_NAMES, stats.cpu().numpy().astype(np.int64).tolist())) if counters else {})


def parity(gpu_paths: np.ndarray, gpu_len: np.ndarray, ora: oracle.WalkResult) -> dict:
    """Free-running comparison of GPU walks with oracle walks from the same inputs.

    A walker is compared up to its first differing slot; that step must be a flagged
    boundary (oracle margin < MARGIN) for the difference to be tolerated.
    """
    L = gpu_paths.shape[1] - 1
    diff = gpu_paths != ora.paths
    bad = np.flatnonzero(diff.any(axis=1) | (gpu_len != ora.lengths))
    steps = int(ora.lengths.sum())
    flagged_steps = int((ora.margins < MARGIN).sum()) if ora.margins is not None else -1
    unflagged, flagged = [], []
    for w in bad:
        cols = np.flatnonzero(diff[w])
        jstep = (int(cols[0]) - 1) if cols.size else int(min(gpu_len[w], ora.lengths[w]))
        jstep = max(0, min(jstep, L - 1))
        m = float(ora.margins[w, jstep]) if ora.margins is not None else 0.0
        (flagged if m < MARGIN else unflagged).append((int(w), jstep, m))
    return {"walkers": int(gpu_paths.shape[0]), "steps": steps, "mismatch_walkers": int(bad.size),
            "unflagged": unflagged, "flagged": flagged, "flagged_steps": flagged_steps}


def assert_parity(rep: dict):
    assert not rep["unflagged"], f"unflagged mismatches (walker, step, margin): {rep['unflagged'][:10]}"
    assert len(rep["flagged"]) <= 1e-5 * max(rep["steps"], 1), f"flagged mismatches: {rep['flagged'][:10]}"


_EDGE_KEYS: dict = {}


def _edge_keys(g: dict):
    """Sorted 64-bit keys src * nv + dst of every CSR entry, cached per graph."""
    k = id(g["col"])
    if k not in _EDGE_KEYS:
        _EDGE_KEYS.clear()
        dev = torch.device("cuda:0")
        nv = int(g["nv"])
        rp = torch.from_numpy(g["row_ptr"]).to(dev)
        col = torch.from_numpy(g["col"]).to(dev).long()
        src = torch.repeat_interleave(torch.arange(nv, device=dev), rp[1:] - rp[:-1])
        _EDGE_KEYS[k] = src * nv + col  # ascending: rows in order, columns sorted
    return _EDGE_KEYS[k]


def edge_check_torch(g: dict, paths: np.ndarray, lengths: np.ndarray):
    """Every step lands on a neighbour (vectorised on the GPU with torch)."""
    dev = torch.device("cuda:0")
    nv = int(g["nv"])
    keys = _edge_keys(g)
    P = torch.from_numpy(paths).to(dev).long()
    ln = torch.from_numpy(lengths).to(dev).long()
    j = torch.arange(P.shape[1] - 1, device=dev)
    taken = j[None, :] < ln[:, None]
    a, b = P[:, :-1][taken], P[:, 1:][taken]
    q = a * nv + b
    pos = torch.searchsorted(keys, q).clamp(max=keys.numel() - 1)
    ok = keys[pos] == q
    pad_ok = (P[:, 1:][~taken] == -1).all()
    return bool(ok.all().item()), bool(pad_ok.item()), (pos, taken)
