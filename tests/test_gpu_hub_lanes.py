"""eRVS with more reservoir lanes on long rows (needs an MI355X).

A plan's degree bucket (hub_deg, hub_lanes) runs the eRVS steps at rows of degree
>= hub_deg with P = hub_lanes reservoir lanes (Section 3.2, parallel form: lane l owns
items l, l + P, l + 2P, ...) and every other step with P = 64.  P changes the random
stream, so the oracle replays each plan with the same bucket; the bar is the one of the
other parity tests (identical walks up to flagged 1e-6 margins, and equal counters when
nothing differs), and a chi-square at the hub against the exact transition.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import GpuGraph, assert_parity, gpu_walk, parity
from tests._helpers import hub_ring_graph
from tests.test_gpu_parity import COUNTERS, N2V, MP, STRATS, _assert_counters, _hub_chisq, _run_both

import paper_2512_00705_amd as fw

pytestmark = pytest.mark.gpu

PR2 = oracle.Logic(kind=oracle.SECOND_PR, weighted=True, gamma=0.2)
LOGICS = {"node2vec": N2V, "secondpr": PR2, "metapath": MP}


@pytest.fixture(scope="module")
def g12():
    return synth.rmat(12, 8 << 12, seed=1, nlabels=5)


@pytest.fixture(scope="module")
def gg12(g12):
    gg = GpuGraph(g12)
    yield gg
    gg.close()


@pytest.mark.parametrize("hub_lanes", [128, 256])
@pytest.mark.parametrize("lds_cap", [2048, 16])
@pytest.mark.parametrize("strategy", ["rvs", "auto"])
def test_hub_lanes_hub_rows(hub_lanes, lds_cap, strategy):
    """A 3000-neighbour hub (scan of 3000 / P rounds) and leaves of degree 3; N(prev) in
    LDS or in global memory; the bucket boundary (>=) at the hub's degree."""
    g = hub_ring_graph(3000)
    gg = GpuGraph(g)
    try:
        starts = np.arange(1, 3001, dtype=np.int32)
        for hub_deg in (1000, 3000, 3001):
            pl = oracle.Plan(rho=1.0, hub_deg=hub_deg, hub_lanes=hub_lanes)
            print("hub rows", hub_lanes, lds_cap, strategy, hub_deg, flush=True)
            p, ln, st, ora = _run_both(gg, g, N2V, pl, STRATS[strategy], starts, 6, 11, lds_cap=lds_cap)
            rep = parity(p, ln, ora)
            assert_parity(rep)
            if rep["mismatch_walkers"] == 0:
                _assert_counters(st, ora)
            if strategy == "rvs":
                assert st["rvs_triggers"] > 0
    finally:
        gg.close()


@pytest.mark.parametrize("logic", list(LOGICS))
@pytest.mark.parametrize("strategy", ["rvs", "auto"])
@pytest.mark.parametrize("hub_lanes", [128, 256])
def test_hub_lanes_scale12(g12, gg12, logic, strategy, hub_lanes):
    """R-MAT scale 12 (rows up to a few hundred entries), bucket at degree 128, all three
    logics; one walker per vertex (MetaPath: 5000 uniform starts)."""
    lg = LOGICS[logic]
    pl = oracle.Plan(rho=2.0, rjs_cap=64, hub_deg=128, hub_lanes=hub_lanes)
    starts = (synth.uniform_starts(g12["nv"], 5000, 42) if logic == "metapath" else synth.all_vertices(g12["nv"]))
    p, ln, st, ora = _run_both(gg12, g12, lg, pl, STRATS[strategy], starts, 20, 42)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)
    # the bucket changes the stream: eRVS-only walks differ from the P = 64 plan's (under
    # AUTO the long rows mostly go to eRJS, and the walks may coincide)
    if strategy == "rvs":
        p64, _, _ = gpu_walk(gg12, lg, oracle.Plan(rho=2.0, rjs_cap=64), STRATS[strategy], starts, 20, 42)
        assert not np.array_equal(p, p64)


@pytest.mark.parametrize("hub_lanes", [128, 256])
def test_hub_lanes_chisquare(hub_lanes):
    """Second step at a 600-neighbour hub from leaf 1 with the hub's eRVS at P = hub_lanes."""
    g = hub_ring_graph(600)
    gg = GpuGraph(g)
    try:
        _hub_chisq(g, gg, N2V, oracle.Plan(rho=1.0, hub_deg=600, hub_lanes=hub_lanes), oracle.RVS_ONLY, 31,
                   f"hub lanes {hub_lanes}")
    finally:
        gg.close()


def test_hub_lanes_argument_errors(g12, gg12):
    lg = fw.fw_logic_node2vec(2.0, 0.5, True)
    dev = torch.device("cuda:0")
    s = torch.zeros(4, dtype=torch.int32, device=dev)
    out = torch.zeros(4 * 6, dtype=torch.int32, device=dev)
    ln = torch.zeros(4, dtype=torch.int32, device=dev)
    for bad in (fw.fw_plan_default(hub_deg=100, hub_lanes=96), fw.fw_plan_default(hub_deg=100, hub_lanes=1024),
                fw.fw_plan_default(hub_deg=-1)):
        with pytest.raises(fw.FlexiWalkError):
            fw.fw_walk(gg12.handle, lg, bad, 0, s, 4, 5, 1, out, ln)
    # batches run P = 64 only
    q = fw.fw_query()
    q.logic, q.n, q.L, q.seed = lg, 4, 5, 1
    q.start_off, q.out_off, q.len_off = 0, 0, 0
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_batch_create(gg12.handle, [q], fw.fw_plan_default(hub_deg=100, hub_lanes=256), fw.FW_AUTO, s, out, ln)
    # hub_deg = 0 switches the bucket off whatever hub_lanes says
    b = fw.fw_batch_create(gg12.handle, [q], fw.fw_plan_default(hub_deg=0, hub_lanes=64), fw.FW_AUTO, s, out, ln)
    fw.fw_batch_destroy(b)
