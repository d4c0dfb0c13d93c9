"""eRVS with the lanes' shared threshold (plan rvs_share = 1; needs an MI355X).

After every scan round in which some lane drew a key, each lane below the largest
threshold takes it and rescales its remaining skip (an extension of the parallel eRVS of
Section 3.2: the remaining skip is exponential, so the rescaled skip is that of the new
threshold).  It changes the random stream, so the oracle replays each plan with the same
setting; the bar is the one of the other parity tests (identical walks up to flagged 1e-6
margins, equal counters when nothing differs), a chi-square at the hub against the exact
transition, and fewer jump events than the paper's form on the same walks.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import GpuGraph, assert_parity, fw_plan, gpu_walk, parity
from tests._helpers import hub_ring_graph
from tests.test_gpu_batch import Batch, _small_batch
from tests.test_gpu_parity import N2V, MP, STRATS, _assert_counters, _hub_chisq, _run_both
from tests.test_gpu_serve import _serve_all

import paper_2512_00705_amd as fw

pytestmark = pytest.mark.gpu

PR2 = oracle.Logic(kind=oracle.SECOND_PR, weighted=True, gamma=0.2)
LOGICS = {"node2vec": N2V, "secondpr": PR2, "metapath": MP}
BUCKETS = {"P64": (0, 64), "hub128": (1000, 128), "hub256": (1000, 256)}


@pytest.fixture(scope="module")
def g12():
    return synth.rmat(12, 8 << 12, seed=1, nlabels=5)


@pytest.fixture(scope="module")
def gg12(g12):
    gg = GpuGraph(g12)
    yield gg
    gg.close()


@pytest.mark.parametrize("bucket", list(BUCKETS))
@pytest.mark.parametrize("lds_cap", [2048, 16])
@pytest.mark.parametrize("strategy", ["rvs", "auto"])
def test_rvs_share_hub_rows(bucket, lds_cap, strategy):
    """A 3000-neighbour hub (47 rounds of 64, or 12 of 256) and leaves of degree 3; N(prev)
    in LDS or in global memory; every walker replayed by the oracle, and fewer jump events
    than the same plan without sharing."""
    g = hub_ring_graph(3000)
    gg = GpuGraph(g)
    try:
        starts = np.arange(1, 3001, dtype=np.int32)
        hub_deg, hub_lanes = BUCKETS[bucket]
        pl = oracle.Plan(rho=1.0, hub_deg=hub_deg, hub_lanes=hub_lanes, rvs_share=True)
        print("share hub rows", bucket, lds_cap, strategy, flush=True)
        p, ln, st, ora = _run_both(gg, g, N2V, pl, STRATS[strategy], starts, 6, 11, lds_cap=lds_cap)
        rep = parity(p, ln, ora)
        assert_parity(rep)
        if rep["mismatch_walkers"] == 0:
            _assert_counters(st, ora)
        if strategy == "rvs":
            paper = oracle.Plan(rho=1.0, hub_deg=hub_deg, hub_lanes=hub_lanes)
            _, _, st0 = gpu_walk(gg, N2V, paper, STRATS[strategy], starts, 6, 11, lds_cap=lds_cap)
            assert 0 < st["rvs_triggers"] < 0.5 * st0["rvs_triggers"], (st["rvs_triggers"], st0["rvs_triggers"])
    finally:
        gg.close()


@pytest.mark.parametrize("logic", list(LOGICS))
@pytest.mark.parametrize("strategy", ["rvs", "auto"])
@pytest.mark.parametrize("bucket", ["P64", "hub256"])
def test_rvs_share_scale12(g12, gg12, logic, strategy, bucket):
    """R-MAT scale 12, all three logics, one walker per vertex (MetaPath: 5000 uniform
    starts), the hub bucket at degree 128 where it applies."""
    lg = LOGICS[logic]
    hub_lanes = BUCKETS[bucket][1]
    pl = oracle.Plan(rho=2.0, rjs_cap=64, hub_deg=128 if hub_lanes > 64 else 0, hub_lanes=hub_lanes,
                     rvs_share=True)
    starts = (synth.uniform_starts(g12["nv"], 5000, 42) if logic == "metapath" else synth.all_vertices(g12["nv"]))
    print("share scale12", logic, strategy, bucket, flush=True)
    p, ln, st, ora = _run_both(gg12, g12, lg, pl, STRATS[strategy], starts, 20, 42)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)


@pytest.mark.parametrize("hub_lanes", [64, 256])
def test_rvs_share_chisquare(hub_lanes):
    """Second step at a 600-neighbour hub from leaf 1, the hub's eRVS sharing thresholds."""
    g = hub_ring_graph(600)
    gg = GpuGraph(g)
    try:
        pl = oracle.Plan(rho=1.0, hub_deg=600 if hub_lanes > 64 else 0, hub_lanes=hub_lanes, rvs_share=True)
        _hub_chisq(g, gg, N2V, pl, oracle.RVS_ONLY, 37, f"shared threshold P={hub_lanes}")
    finally:
        gg.close()


def test_rvs_share_batch(g12, gg12):
    """A batch of 40 Node2Vec queries (each its own p, q, L, seed) under eRVS-only with the
    shared threshold: every query equals the oracle's walks."""
    qd = _small_batch(g12["nv"], 40, 5)
    logics = [oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=float(qd["p"][i]), q=float(qd["q"][i]))
              for i in range(40)]
    pl = oracle.Plan(rho=4.0, rvs_share=True)
    b = Batch(gg12, qd, [fw.fw_logic_node2vec(l.p, l.q, True) for l in logics], fw_plan(pl), oracle.RVS_ONLY)
    try:
        fw.fw_batch_launch(b.h, b.stats)
        og = oracle.Graph(g12)
        for i in range(40):
            n = int(qd["n"][i])
            if n == 0:
                continue
            p, ln = b.query(i)
            st = qd["starts"][qd["start_off"][i]:qd["start_off"][i] + n]
            ora = oracle.walk(og, logics[i], pl, oracle.RVS_ONLY, st, int(qd["L"][i]), int(qd["seed"][i]))
            assert_parity(parity(p, ln, ora))
    finally:
        b.close()


def test_rvs_share_served(g12, gg12):
    """Served walks suspended every 3 steps, eRVS-only with the shared threshold, equal
    the oracle's."""
    pl = oracle.Plan(rho=1.0, rjs_cap=64, rvs_share=True)
    rng = np.random.default_rng(13)
    reqs = [(oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=float(rng.choice([0.25, 2.0])), q=2.0),
             rng.integers(0, g12["nv"], int(rng.integers(1, 300))).astype(np.int32), int(rng.integers(1, 25)), 900 + i)
            for i in range(10)]
    srv = fw.fw_server_create(gg12.handle, fw_plan(pl), fw.FW_RVS_ONLY, 64 << 20, tick_steps=3, max_active=8)
    try:
        results = _serve_all(srv, reqs)
    finally:
        fw.fw_server_destroy(srv)
    og = oracle.Graph(g12)
    for k, (lg, st, L, seed) in enumerate(reqs):
        p, ln, _ = results[k]
        assert_parity(parity(p, ln, oracle.walk(og, lg, pl, oracle.RVS_ONLY, st, L, seed)))


def test_rvs_share_argument_errors(gg12):
    lg = fw.fw_logic_node2vec(2.0, 0.5, True)
    dev = torch.device("cuda:0")
    s = torch.zeros(4, dtype=torch.int32, device=dev)
    out = torch.zeros(4 * 6, dtype=torch.int32, device=dev)
    ln = torch.zeros(4, dtype=torch.int32, device=dev)
    for bad in (2, -1):
        with pytest.raises(fw.FlexiWalkError):
            fw.fw_walk(gg12.handle, lg, fw.fw_plan_default(rvs_share=bad), 0, s, 4, 5, 1, out, ln)
