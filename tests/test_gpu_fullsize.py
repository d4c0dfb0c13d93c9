"""Full-size workloads on the GPU, checked on sampled walkers and by invariants.

Scale-22 R-MAT (4.19M vertices, ~128M CSR entries, weights U(1,10), labels 0..4):
* Node2Vec p=0.5 q=2.0, one walker per vertex, L=80, in the launch configuration the
  benchmark times (default plan, autotuned rho), for AUTO, eRVS-only and eRJS-only;
* MetaPath schema (0,1,2,3,4) repeated, 1M uniform starts (seed 42), L=40.
The oracle replays a seeded sample of walkers (same walker ids, so the same random
streams; every walker for MetaPath) and every walk of the launch is checked to step along
edges, to match the schema, and to pad with -1.  Also at full size: 4096 batched queries
on the skewed scale-24 graph, and the walk server on the labelled scale-25 graph.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import GpuGraph, assert_parity, edge_check_torch, gpu_walk, parity

import paper_2512_00705_amd as fw

pytestmark = pytest.mark.gpu

N2V = oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=0.5, q=2.0)
MP = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2, 3, 4))


@pytest.fixture(scope="module")
def g22():
    return synth.cached("rmat22_labels")


@pytest.fixture(scope="module")
def gg22(g22):
    gg = GpuGraph(g22, index=True, alias=True, label_alias=True)  # as the benchmark runs it
    yield gg
    gg.close()


@pytest.fixture(scope="module")
def og22(g22):
    og = oracle.Graph(g22)
    og.aux()
    return og


@pytest.fixture(scope="module")
def tuned22(gg22):
    return fw.fw_plan_autotune(gg22.handle, fw.fw_logic_node2vec(0.5, 2.0, True))


def test_alias_tables_scale22(g22, gg22, og22):
    """The scale-22 proposal records' alias tables (128M entries, rows up to 163,520
    entries) equal the oracle's sweep entry for entry."""
    print("exporting the GPU tables", flush=True)
    thr, al = fw.fw_graph_export_alias(gg22.handle, gg22.ne)
    print("oracle sweep", flush=True)
    othr, oal = og22.alias()
    assert np.array_equal(al, oal), int(np.count_nonzero(al != oal))
    assert np.array_equal(thr, othr), int(np.count_nonzero(thr != othr))


def _sample(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(k, n), replace=False)).astype(np.int64)


@pytest.mark.parametrize("strategy,k,bound,proposal,rho", [
    (oracle.AUTO, 65536, None, None, None), (oracle.RJS_ONLY, 65536, None, None, None),
    (oracle.RVS_ONLY, 16384, None, None, None), (oracle.AUTO, 65536, 0, 0, None), (oracle.AUTO, 65536, 1, 0, None),
    (oracle.RJS_ONLY, 65536, 1, 1, None), (oracle.AUTO, 65536, 2, 0, None), (oracle.RJS_ONLY, 65536, 2, 1, None),
    (oracle.AUTO, 65536, 0, 0, 8.0)],
    ids=["auto", "rjs", "rvs", "auto_paper", "auto_split_uniform", "rjs_split_h_proposals", "auto_member_uniform",
         "rjs_member_h_proposals", "auto_paper_mixed"])
def test_node2vec_scale22(g22, gg22, og22, tuned22, strategy, k, bound, proposal, rho):
    """None: the autotuned plan as the benchmark runs it; otherwise that plan with the
    bound (paper's / split / member board), the proposal (uniform / h-proportional) and the
    cost ratio rho forced.  With the paper's board at rho = 8 the cost model of Eq. (runtime)
    sends the steps at low-degree vertices to eRVS and the others to eRJS, so both kernels
    run in one full-size job."""
    tuned = tuned22
    pl = oracle.Plan(rho=tuned.rho if rho is None else rho, d_lo=tuned.d_lo, rjs_cap=tuned.rjs_cap,
                     bound=tuned.bound if bound is None else bound,
                     proposal=tuned.proposal if proposal is None else proposal, hub_deg=tuned.hub_deg,
                     hub_lanes=tuned.hub_lanes, rvs_share=bool(tuned.rvs_share))
    starts = synth.all_vertices(g22["nv"])
    p, ln, st = gpu_walk(gg22, N2V, pl, strategy, starts, 80, 42)
    # the launch the benchmark times (no counter array, the counter-free kernel variant)
    # walks exactly as the counted one
    p2, ln2, _ = gpu_walk(gg22, N2V, pl, strategy, starts, 80, 42, counters=False)
    assert np.array_equal(p, p2) and np.array_equal(ln, ln2)
    del p2, ln2
    ok, pad_ok, _ = edge_check_torch(g22, p, ln)
    assert ok and pad_ok
    deg = np.diff(g22["row_ptr"])
    assert ((ln == 80) == (deg > 0)).all()  # undirected: only isolated starts stop early
    sub = _sample(g22["nv"], k, 1234)
    ora = oracle.walk(og22, N2V, pl, strategy, starts[sub], 80, 42, walker_ids=sub)
    rep = parity(p[sub], ln[sub], ora)
    print("scale22", strategy, {k2: (v if not isinstance(v, list) else len(v)) for k2, v in rep.items()}, st)
    assert_parity(rep)
    assert rep["steps"] >= min(k, 65536) * 40
    if rho is not None:
        assert st["rjs_steps"] > 0 and st["rvs_steps"] > 0, st
        assert (ora.kinds == 0).any() and (ora.kinds == 1).any()


@pytest.mark.parametrize("hub_deg,hub_lanes,share", [(1024, 256, False), (4096, 128, False), (0, 64, True),
                                                     (1024, 256, True)])
def test_node2vec_scale22_hub_lanes(g22, gg22, og22, tuned22, hub_deg, hub_lanes, share):
    """eRVS-only at scale 22 with P = hub_lanes on rows of degree >= hub_deg (a third of the
    steps, most of the scanned entries), and with the lanes' shared threshold: 16,384
    sampled walkers against the oracle with the same degree bucket and sharing."""
    pl = oracle.Plan(rho=tuned22.rho, d_lo=tuned22.d_lo, rjs_cap=tuned22.rjs_cap, bound=tuned22.bound,
                     proposal=tuned22.proposal, hub_deg=hub_deg, hub_lanes=hub_lanes, rvs_share=share)
    starts = synth.all_vertices(g22["nv"])
    p, ln, st = gpu_walk(gg22, N2V, pl, oracle.RVS_ONLY, starts, 80, 42, counters=False)
    ok, pad_ok, _ = edge_check_torch(g22, p, ln)
    assert ok and pad_ok
    sub = _sample(g22["nv"], 16384, 1234)
    ora = oracle.walk(og22, N2V, pl, oracle.RVS_ONLY, starts[sub], 80, 42, walker_ids=sub)
    rep = parity(p[sub], ln[sub], ora)
    print("scale22 hub lanes", hub_deg, hub_lanes, share, {k2: (v if not isinstance(v, list) else len(v))
                                                    for k2, v in rep.items()})
    assert_parity(rep)
    assert rep["steps"] >= 16384 * 40


@pytest.mark.parametrize("bound", [None, 0], ids=["tuned", "paper"])
def test_second_pr_scale22(g22, gg22, og22, bound):
    """Second-order PageRank (gamma = 0.2), one walker per vertex, L = 80, the autotuned
    plan (the member board where it wins) and the paper's bound; sampled walkers replayed
    by the oracle, every walk checked to follow edges."""
    lg = oracle.Logic(kind=oracle.SECOND_PR, weighted=True, gamma=0.2)
    tuned = fw.fw_plan_autotune(gg22.handle, fw.fw_logic_second_pr(0.2, True))
    pl = oracle.Plan(rho=tuned.rho, d_lo=tuned.d_lo, rjs_cap=tuned.rjs_cap,
                     bound=tuned.bound if bound is None else bound, proposal=tuned.proposal,
                     hub_deg=tuned.hub_deg, hub_lanes=tuned.hub_lanes, rvs_share=bool(tuned.rvs_share))
    starts = synth.all_vertices(g22["nv"])
    p, ln, st = gpu_walk(gg22, lg, pl, oracle.AUTO, starts, 80, 42)
    p2, ln2, _ = gpu_walk(gg22, lg, pl, oracle.AUTO, starts, 80, 42, counters=False)
    assert np.array_equal(p, p2) and np.array_equal(ln, ln2)
    del p2, ln2
    ok, pad_ok, _ = edge_check_torch(g22, p, ln)
    assert ok and pad_ok
    sub = _sample(g22["nv"], 16384, 4321)
    ora = oracle.walk(og22, lg, pl, oracle.AUTO, starts[sub], 80, 42, walker_ids=sub)
    rep = parity(p[sub], ln[sub], ora)
    print("secondpr22", pl, {k2: (v if not isinstance(v, list) else len(v)) for k2, v in rep.items()}, st)
    assert_parity(rep)


def test_node2vec_scale22_h8(g22):
    """The scale-22 Node2Vec job with the weights stored as 8-bit codes (4-byte edge
    records): the autotuned plan and eRVS-only, sampled walkers replayed by the oracle on
    the same codes, every walk checked to follow edges."""
    codes, scale = synth.quantize_u8(g22["h"])
    gq = dict(g22, h=None, h8=codes, h_scale=scale)
    gg = GpuGraph(gq, index=True, alias=True)
    try:
        tuned = fw.fw_plan_autotune(gg.handle, fw.fw_logic_node2vec(0.5, 2.0, True))
        og = oracle.Graph(gq)
        og.aux()
        starts = synth.all_vertices(g22["nv"])
        for strategy, k in ((oracle.AUTO, 65536), (oracle.RVS_ONLY, 16384)):
            pl = oracle.Plan(rho=tuned.rho, d_lo=tuned.d_lo, rjs_cap=tuned.rjs_cap, bound=tuned.bound,
                             proposal=tuned.proposal, hub_deg=tuned.hub_deg, hub_lanes=tuned.hub_lanes,
                             rvs_share=bool(tuned.rvs_share))
            p, ln, st = gpu_walk(gg, N2V, pl, strategy, starts, 80, 42)
            ok, pad_ok, _ = edge_check_torch(g22, p, ln)
            assert ok and pad_ok
            sub = _sample(g22["nv"], k, 777)
            ora = oracle.walk(og, N2V, pl, strategy, starts[sub], 80, 42, walker_ids=sub)
            rep = parity(p[sub], ln[sub], ora)
            print("h8 scale22", strategy, {k2: (v if not isinstance(v, list) else len(v)) for k2, v in rep.items()},
                  st)
            assert_parity(rep)
    finally:
        gg.close()


@pytest.mark.parametrize("proposal", [None, 2], ids=["tuned", "label_groups"])
def test_metapath_scale22(g22, gg22, og22, proposal):
    """The MetaPath job at full size with the tuned plan, and with label-conditioned
    proposals forced; every walker replayed by the oracle."""
    tuned = fw.fw_plan_autotune(gg22.handle, fw.fw_logic_metapath([0, 1, 2, 3, 4], True))
    pl = oracle.Plan(rho=tuned.rho, d_lo=tuned.d_lo, rjs_cap=tuned.rjs_cap, hub_deg=tuned.hub_deg,
                     hub_lanes=tuned.hub_lanes, proposal=tuned.proposal if proposal is None else proposal,
                     rvs_share=bool(tuned.rvs_share))
    starts = synth.uniform_starts(g22["nv"], 1 << 20, 42)
    p, ln, st = gpu_walk(gg22, MP, pl, oracle.AUTO, starts, 40, 42)
    ok, pad_ok, (pos, taken) = edge_check_torch(g22, p, ln)
    assert ok and pad_ok
    # schema: the label of the edge taken at step j is schema[j mod 5]
    lab = torch.from_numpy(g22["label"]).to(pos.device)
    jj = torch.arange(40, device=pos.device)[None, :].expand(taken.shape[0], 40)[taken]
    assert bool((lab[pos] == (jj % 5).to(lab.dtype)).all().item())
    assert st["ended_early"] > 0
    # every walker of the job replayed by the oracle
    ora = oracle.walk(og22, MP, pl, oracle.AUTO, starts, 40, 42)
    rep = parity(p, ln, ora)
    print("metapath22", pl, {k2: (v if not isinstance(v, list) else len(v)) for k2, v in rep.items()}, st)
    assert_parity(rep)
    if pl.proposal == 2:
        assert st["rjs_trials"] == st["rjs_steps"] > 0


def test_batched_scale24():
    """4096 Node2Vec queries (p, q from {0.25..4}, start sets log-uniform 1..65536, L in
    5..200) on the skewed scale-24 R-MAT in one launch; 32 queries replayed by the oracle
    on up to 256 walkers each, and every walk of 256 queries checked to follow edges."""
    g = synth.cached("rmat24_skew")
    gg = GpuGraph(g, index=True, alias=True)
    try:
        qd = synth.batch_queries(g["nv"], 4096, 7)
        dev = torch.device("cuda:0")
        starts = torch.from_numpy(qd["starts"]).to(dev)
        paths = torch.full((qd["total_paths"],), -7, dtype=torch.int32, device=dev)
        lengths = torch.full((int(qd["n"].sum()),), -7, dtype=torch.int32, device=dev)
        stats = torch.zeros(fw.FW_NSTATS, dtype=torch.int64, device=dev)
        tuned = fw.fw_plan_autotune(gg.handle, fw.fw_logic_node2vec(1.0, 1.0, True))
        pl = oracle.Plan(rho=tuned.rho, d_lo=tuned.d_lo, rjs_cap=tuned.rjs_cap, bound=tuned.bound,
                         proposal=tuned.proposal, rvs_share=bool(tuned.rvs_share))
        qs = []
        for i in range(4096):
            q = fw.fw_query()
            q.logic = fw.fw_logic_node2vec(float(qd["p"][i]), float(qd["q"][i]), True)
            q.n, q.L, q.seed = int(qd["n"][i]), int(qd["L"][i]), int(qd["seed"][i])
            q.start_off, q.out_off, q.len_off = int(qd["start_off"][i]), int(qd["out_off"][i]), int(qd["len_off"][i])
            qs.append(q)
        b = fw.fw_batch_create(gg.handle, qs, tuned, fw.FW_AUTO, starts, paths, lengths)
        fw.fw_batch_launch(b, stats)
        fw.fw_graph_check(gg.handle)
        torch.cuda.synchronize()
        fw.fw_batch_destroy(b)
        st = stats.cpu().numpy()
        print("batched24", dict(zip(fw.STAT_NAMES, st.tolist())))
        og = oracle.Graph(g)
        og.aux()
        rng = np.random.default_rng(5)
        order = np.argsort(qd["n"])
        picks = np.concatenate([order[:8], order[2040:2048], order[-16:]])
        steps = 0
        for i in picks:
            n, L = int(qd["n"][i]), int(qd["L"][i])
            o = int(qd["out_off"][i])
            sub = np.sort(rng.choice(n, size=min(n, 256), replace=False)).astype(np.int64)
            p = paths[o:o + n * (L + 1)].view(n, L + 1)[torch.from_numpy(sub).to(dev)].cpu().numpy()
            ln = lengths[int(qd["len_off"][i]):int(qd["len_off"][i]) + n][torch.from_numpy(sub).to(dev)].cpu().numpy()
            st_q = qd["starts"][qd["start_off"][i]:qd["start_off"][i] + n][sub]
            lg = oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=float(qd["p"][i]), q=float(qd["q"][i]))
            ora = oracle.walk(og, lg, pl, oracle.AUTO, st_q, L, int(qd["seed"][i]), walker_ids=sub)
            rep = parity(p, ln, ora)
            assert_parity(rep)
            steps += rep["steps"]
        assert steps > 10000
        for i in rng.choice(4096, 256, replace=False):
            n, L = int(qd["n"][i]), int(qd["L"][i])
            o = int(qd["out_off"][i])
            p = paths[o:o + n * (L + 1)].view(n, L + 1).cpu().numpy()
            ln = lengths[int(qd["len_off"][i]):int(qd["len_off"][i]) + n].cpu().numpy()
            ok, pad_ok, _ = edge_check_torch(g, p, ln)
            assert ok and pad_ok, i
    finally:
        gg.close()


def test_served_scale25():
    """The served configuration at full size: R-MAT scale 25 with labels (1.05 B entries,
    rows up to 639,407), edge index and proposal records built, one plan tuned over the
    served logic mix (Node2Vec p, q in {0.25, 0.5, 1, 2, 4}, MetaPath (0,1,2,3,4)), continuous
    batching with 64-step ticks and a 32 GiB budget.  48 requests (start sets log-uniform in
    1..4096, L in 10..100) arrive together; up to 64 walkers of every request are replayed
    by the oracle."""
    from tests._gpu import fw_plan
    from tests.test_gpu_serve import _serve_all

    print("generating R-MAT scale 25", flush=True)
    g = synth.workload_graph("rmat25_labels")
    print("uploading and building the edge index and proposal records", flush=True)
    gg = GpuGraph(g, index=True, alias=True)
    try:
        pq = [0.25, 0.5, 1.0, 2.0, 4.0]
        mix = [fw.fw_logic_node2vec(p, q, True) for p in pq for q in pq]
        mix.append(fw.fw_logic_metapath([0, 1, 2, 3, 4], True))
        tuned = fw.fw_plan_autotune_mix(gg.handle, mix)
        pl = oracle.Plan(rho=tuned.rho, d_lo=tuned.d_lo, rjs_cap=tuned.rjs_cap, bound=tuned.bound,
                         proposal=tuned.proposal, rvs_share=bool(tuned.rvs_share))
        print("plan", tuned.rho, tuned.d_lo, tuned.lds_cap, tuned.bound, tuned.proposal, tuned.rjs_cap, flush=True)
        rng = np.random.default_rng(25)
        reqs = []
        for i in range(48):
            if i % 2 == 0:
                lg = oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=float(rng.choice(pq)), q=float(rng.choice(pq)))
            else:
                lg = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2, 3, 4))
            n = int(np.clip(np.floor(np.exp(rng.uniform(0, np.log(4096)))), 1, 4096))
            reqs.append((lg, rng.integers(0, g["nv"], n).astype(np.int32), int(rng.integers(10, 101)), 5000 + i))
        srv = fw.fw_server_create(gg.handle, fw_plan(pl, lds_cap=tuned.lds_cap, grid=tuned.grid), fw.FW_AUTO,
                                  32 << 30, tick_steps=64, max_active=8192, max_pending=1 << 16)
        try:
            print("serving", flush=True)
            results = _serve_all(srv, reqs)
            stats = fw.fw_server_stats(srv)
        finally:
            fw.fw_server_destroy(srv)
        assert len(results) == len(reqs) and stats["finished"] == len(reqs) and stats["bytes_in_use"] == 0
        print("oracle replay", flush=True)
        og = oracle.Graph(g)
        og.aux()
        steps = 0
        for k, (lg, st, L, seed) in enumerate(reqs):
            p, ln, _ = results[k]
            sub = np.arange(min(64, len(st)), dtype=np.int64)
            ora = oracle.walk(og, lg, pl, oracle.AUTO, st[sub], L, seed, walker_ids=sub)
            rep = parity(p[sub], ln[sub], ora)
            assert_parity(rep)
            steps += rep["steps"]
        print("served scale 25: requests", len(reqs), "oracle steps", steps, stats, flush=True)
    finally:
        gg.close()
