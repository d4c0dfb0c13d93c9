"""A graph of more than 2^32 CSR entries on the GPU: 64-bit row starts.

Circulant graph: vertex v is joined to v +- 1 .. v +- 2048 (mod nv) with nv = 2^20 + 2^16,
so every degree is 4096, ne = 4096 * nv (about 4.56e9, beyond 2^32), and the rows of
v >= 2^20 start at or beyond 2^32: their starts need the high bits the device keeps beside
the 32-bit vertex records.  Unweighted (h = 1), so the graph takes 18 GB of col, 37 GB of
edge records and an 18 GB host copy for the oracle.  Rows are built on the device and
sorted there; the oracle replays every walker of each launch (same walker ids, so the
same random streams), half of them started in the wide region.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from tests._gpu import GpuGraph, assert_parity, gpu_walk, parity

pytestmark = pytest.mark.gpu

HALF = 2048
D = 2 * HALF
NV = (1 << 20) + (1 << 16)
NE = NV * D
N2V = oracle.Logic(kind=oracle.NODE2VEC, weighted=False, p=0.5, q=2.0)
PR2 = oracle.Logic(kind=oracle.SECOND_PR, weighted=False, gamma=0.2)


def _circulant(dev) -> tuple[torch.Tensor, torch.Tensor]:
    offs = torch.cat([torch.arange(-HALF, 0), torch.arange(1, HALF + 1)]).to(dev)
    col = torch.empty(NE, dtype=torch.int32, device=dev)
    step = 1 << 16
    for v0 in range(0, NV, step):
        v = torch.arange(v0, min(NV, v0 + step), device=dev)
        rows = torch.remainder(v[:, None] + offs[None, :], NV)
        col[v0 * D:(v0 + v.numel()) * D] = torch.sort(rows, dim=1).values.reshape(-1).to(torch.int32)
        del rows
    row_ptr = torch.arange(NV + 1, dtype=torch.int64, device=dev) * D
    return row_ptr, col


@pytest.fixture(scope="module")
def wide():
    dev = torch.device("cuda:0")
    row_ptr, col = _circulant(dev)
    torch.cuda.synchronize()
    g = {"nv": NV, "ne": NE, "row_ptr": row_ptr.cpu().numpy(), "col": col.cpu().numpy(), "h": None, "label": None}
    del col, row_ptr
    torch.cuda.empty_cache()
    assert g["row_ptr"][-1] == NE and NE >= (1 << 32)
    gg = GpuGraph(g, on_device=False)  # uploaded from the host copy; preprocessed, no index or records
    og = oracle.Graph(g)
    og.aux()
    yield g, gg, og
    gg.close()
    torch.cuda.empty_cache()


def _starts(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    hi = rng.integers(1 << 20, NV, n // 2)  # rows that start beyond 2^32
    lo = rng.integers(0, NV, n - n // 2)
    return np.concatenate([hi, lo]).astype(np.int32)


def _steps_ok(p: np.ndarray, ln: np.ndarray) -> bool:
    """Every taken step joins two vertices at circular distance 1..2048; padding is -1."""
    j = np.arange(p.shape[1] - 1)
    taken = j[None, :] < ln[:, None]
    a, b = p[:, :-1][taken].astype(np.int64), p[:, 1:][taken].astype(np.int64)
    d = (b - a) % NV
    return bool((((d >= 1) & (d <= HALF)) | ((d >= NV - HALF) & (d <= NV - 1))).all()
                and (p[:, 1:][~taken] == -1).all())


@pytest.mark.parametrize("lg,strategy,bound,n,speed", [
    (N2V, oracle.AUTO, 0, 4096, {}),
    (N2V, oracle.AUTO, 2, 4096, {"lds_cap": 8192}),
    (N2V, oracle.RVS_ONLY, 0, 1024, {}),
    (PR2, oracle.AUTO, 2, 4096, {})],
    ids=["node2vec_auto", "node2vec_member_board_staged", "node2vec_rvs", "secondpr_member_board"])
def test_wide_graph(wide, lg, strategy, bound, n, speed):
    g, gg, og = wide
    pl = oracle.Plan(bound=bound)
    starts = _starts(n, 11 + bound)
    L = 24
    p, ln, st = gpu_walk(gg, lg, pl, strategy, starts, L, 77, **speed)
    assert (ln == L).all()  # no dead ends: every degree is 4096
    assert _steps_ok(p, ln)
    ora = oracle.walk(og, lg, pl, strategy, starts, L, 77)
    rep = parity(p, ln, ora)
    print("wide", lg.kind, strategy, bound, {k: (v if not isinstance(v, list) else len(v)) for k, v in rep.items()}, st)
    assert_parity(rep)
    # the launch really walked rows that start beyond 2^32
    assert (p[: n // 2, 1:] >= (1 << 20)).any()
