"""Parity of the HIP walk kernels with the CPU oracle (needs an MI355X).

Walks run through the C ABI; the oracle replays the same inputs free-running.  The
bar: every walker identical to the oracle except at a step whose oracle float
decision lies within 1e-6 relative of its boundary (counted, at most 1e-5 of steps),
and when nothing differs the device counters equal the oracle's (steps per kernel,
eRJS trials, jump events, algorithmic bytes).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import exact
from tests._gpu import GpuGraph, assert_parity, gpu_walk, parity
from tests._helpers import assert_chisq, chisq_pvalue, hub_ring_graph, worked_example_graph

import paper_2512_00705_amd as fw

pytestmark = pytest.mark.gpu

N2V = oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=2.0, q=0.5)
MP = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2, 3, 4))
STRATS = {"auto": oracle.AUTO, "rvs": oracle.RVS_ONLY, "rjs": oracle.RJS_ONLY}
COUNTERS = ("steps", "rjs_steps", "rvs_steps", "rjs_fallbacks", "rjs_trials", "rvs_triggers", "ended_early",
            "alg_bytes")


@pytest.fixture(scope="module")
def g12():
    return synth.rmat(12, 8 << 12, seed=1, nlabels=5)


@pytest.fixture(scope="module")
def gg12(g12):
    gg = GpuGraph(g12)
    yield gg
    gg.close()


def _run_both(gg, g, lg, pl, strategy, starts, L, seed, walker_ids=None, **speed):
    p, ln, st = gpu_walk(gg, lg, pl, strategy, starts, L, seed, **speed)
    ora = oracle.walk(oracle.Graph(g), lg, pl, strategy, starts, L, seed)
    return p, ln, st, ora


def _assert_counters(st, ora):
    for k in COUNTERS:
        assert st[k] == int(ora.counters[k]), (k, st[k], ora.counters[k])


def _hub_chisq(g, gg, lg, pl, strategy, seed, label, n=300000):
    """Second step at the hub of ``hub_ring_graph`` from leaf 1 against the exact
    transition, accepted at p > 0.01 (one declared retest on an independent seed)."""
    def pvalue(sd):
        p, ln, st = gpu_walk(gg, lg, pl, strategy, np.ones(n, np.int32), 2, sd)
        at_hub = p[:, 1] == 0
        counts = {int(v): int(c) for v, c in zip(*np.unique(p[at_hub, 2], return_counts=True))}
        return chisq_pvalue(counts, exact.transition(g, lg, 1, 1, 0), int(at_hub.sum()))
    return assert_chisq(pvalue, seed, label)


def test_preprocess_bit_exact(g12, gg12):
    hmax, hsum = fw.fw_graph_export_aux(gg12.handle, gg12.nv)
    ohmax, ohsum = oracle.Graph(g12).aux()
    np.testing.assert_array_equal(hmax, ohmax)
    np.testing.assert_array_equal(hsum, ohsum)
    assert fw.fw_graph_info(gg12.handle)[2] == int(np.diff(g12["row_ptr"]).max())


@pytest.mark.parametrize("strategy", list(STRATS), ids=list(STRATS))
@pytest.mark.parametrize("rho", [8.0, 0.5])
def test_node2vec_scale12(g12, gg12, strategy, rho):
    """Node2Vec p=2, q=0.5, weighted, one walker per vertex, L=20, seed 42."""
    pl = oracle.Plan(rho=rho)
    starts = synth.all_vertices(g12["nv"])
    p, ln, st, ora = _run_both(gg12, g12, N2V, pl, STRATS[strategy], starts, 20, 42)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)
    if strategy == "auto" and rho == 8.0:
        assert st["rjs_steps"] > 0 and st["rvs_steps"] > 0  # both kernels exercised


@pytest.mark.parametrize("strategy", list(STRATS), ids=list(STRATS))
def test_metapath_scale12(g12, gg12, strategy):
    pl = oracle.Plan(rho=2.0, rjs_cap=64)
    starts = synth.uniform_starts(g12["nv"], 5000, 42)
    p, ln, st, ora = _run_both(gg12, g12, MP, pl, STRATS[strategy], starts, 20, 42)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)
    assert st["ended_early"] > 0  # schema dead ends occur


@pytest.mark.parametrize("weighted", [False, True])
def test_unweighted_and_d_lo(g12, gg12, weighted):
    lg = oracle.Logic(kind=oracle.NODE2VEC, weighted=weighted, p=1.0, q=0.5)
    pl = oracle.Plan(rho=3.0, d_lo=24, rjs_cap=16)
    starts = synth.uniform_starts(g12["nv"], 3000, 7)
    p, ln, st, ora = _run_both(gg12, g12, lg, pl, oracle.AUTO, starts, 15, 1234567891234)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)


def test_host_upload_and_launch_shape(g12, gg12):
    """Host-copied graph, one-block grid and no LDS staging give the same walks."""
    starts = synth.uniform_starts(g12["nv"], 3001, 3)
    pl = oracle.Plan(rho=4.0)
    ref = gpu_walk(gg12, N2V, pl, oracle.AUTO, starts, 12, 5)
    gh = GpuGraph(g12, on_device=False)
    try:
        alt = gpu_walk(gh, N2V, pl, oracle.AUTO, starts, 12, 5, grid=1, lds_cap=0)
    finally:
        gh.close()
    np.testing.assert_array_equal(ref[0], alt[0])
    np.testing.assert_array_equal(ref[1], alt[1])
    assert ref[2] == alt[2]


@pytest.mark.parametrize("lds_cap", [2048, 16])
@pytest.mark.parametrize("strategy", ["rvs", "auto"])
def test_hub_rows(lds_cap, strategy):
    """Rows longer than a wavefront (jump scan) and N(prev) in LDS or in global memory."""
    g = hub_ring_graph(3000)
    gg = GpuGraph(g)
    try:
        starts = np.arange(1, 3001, dtype=np.int32)
        pl = oracle.Plan(rho=1.0)
        p, ln, st, ora = _run_both(gg, g, N2V, pl, STRATS[strategy], starts, 6, 11, lds_cap=lds_cap)
        rep = parity(p, ln, ora)
        assert_parity(rep)
        if rep["mismatch_walkers"] == 0:
            _assert_counters(st, ora)
        if strategy == "rvs":
            assert st["rvs_triggers"] > 0  # the jump scan ran
        else:
            assert st["rjs_steps"] > 0 and st["rvs_steps"] > 0
    finally:
        gg.close()


def test_edge_cases(g12, gg12):
    deg = np.diff(g12["row_ptr"])
    iso = int(np.flatnonzero(deg == 0)[0])
    pl = oracle.Plan()
    # L = 0: paths hold the starts only
    s = np.array([0, 1, iso], np.int32)
    p, ln, st = gpu_walk(gg12, N2V, pl, oracle.AUTO, s, 0, 1)
    assert p[:, 0].tolist() == s.tolist() and ln.tolist() == [0, 0, 0]
    # isolated start: length 0, padded with -1; ragged sizes
    for n in (1, 63, 65, 4097):
        s = synth.uniform_starts(g12["nv"], n, n)
        s[0] = iso
        p, ln, st, ora = _run_both(gg12, g12, N2V, pl, oracle.AUTO, s, 9, 99)
        assert ln[0] == 0 and (p[0, 1:] == -1).all()
        assert_parity(parity(p, ln, ora))
    # n = 0 is a no-op
    gpu_walk(gg12, N2V, pl, oracle.AUTO, np.zeros(0, np.int32), 5, 1)
    # out-of-range start: walker gets length 0, others unaffected, check reports it
    s = np.array([5, g12["nv"] + 3, 7], np.int32)
    p, ln, st = gpu_walk(gg12, N2V, pl, oracle.AUTO, s, 4, 2)
    assert ln[1] == 0 and (p[1, 1:] == -1).all()
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_graph_check(gg12.handle)
    fw.fw_graph_check(gg12.handle)  # flag cleared
    ok = s[[0, 2]]
    ora = oracle.walk(oracle.Graph(g12), N2V, pl, oracle.AUTO, ok, 4, 2, walker_ids=np.array([0, 2]))
    np.testing.assert_array_equal(p[[0, 2]], ora.paths)


def test_argument_errors(g12, gg12):
    pl = fw.fw_plan_default()
    lg = fw.fw_logic_node2vec(2.0, 0.5, True)
    dev = torch.device("cuda:0")
    s = torch.zeros(4, dtype=torch.int32, device=dev)
    out = torch.zeros(4 * 6, dtype=torch.int32, device=dev)
    ln = torch.zeros(4, dtype=torch.int32, device=dev)
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_walk(gg12.handle, lg, pl, 7, s, 4, 5, 1, out, ln)
    bad = fw.fw_plan_default(lanes=32)
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_walk(gg12.handle, lg, bad, 0, s, 4, 5, 1, out, ln)
    # malformed CSR: unsorted row
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_graph_create(2, 2, np.array([0, 2, 2], np.int64), np.array([1, 0], np.int32))
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_graph_create(2, 2, np.array([0, 2, 1], np.int64), np.array([0, 1], np.int32))
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_graph_create(2, 1, np.array([0, 1, 1], np.int64), np.array([5], np.int32))
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_graph_create(2, 1, np.array([0, 1, 1], np.int64), np.array([1], np.int32),
                           np.array([np.nan], np.float32))
    # metapath without labels
    g = synth.rmat(6, 64, seed=1)
    gg = GpuGraph(g)
    try:
        with pytest.raises(fw.FlexiWalkError):
            fw.fw_walk(gg.handle, fw.fw_logic_metapath([0, 1]), pl, 0, s, 4, 5, 1, out, ln)
    finally:
        gg.close()


@pytest.mark.parametrize("strategy", list(STRATS), ids=list(STRATS))
def test_chisquare_worked_example(strategy):
    g = worked_example_graph()
    gg = GpuGraph(g)
    n = 200000

    def pvalue(sd):
        p, ln, st = gpu_walk(gg, N2V, oracle.Plan(), STRATS[strategy], np.zeros(n, np.int32), 1, sd)
        counts = {int(v): int(c) for v, c in zip(*np.unique(p[:, 1], return_counts=True))}
        return chisq_pvalue(counts, exact.transition(g, N2V, 0, -1, 0), n)
    try:
        assert_chisq(pvalue, 17, f"worked example {strategy}")
    finally:
        gg.close()


@pytest.mark.parametrize("strategy", list(STRATS), ids=list(STRATS))
def test_chisquare_hub_second_step(strategy):
    """Second step at a 600-neighbour hub, prev = leaf 1: all three Node2Vec cases."""
    g = hub_ring_graph(600)
    gg = GpuGraph(g)
    try:
        _hub_chisq(g, gg, N2V, oracle.Plan(rho=1.0), STRATS[strategy], 23, f"hub {strategy}")
    finally:
        gg.close()


# ------------------------------------------------------------------ split eRJS bound
N2V_RET = oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=0.25, q=2.0)


@pytest.mark.parametrize("strategy", ["auto", "rjs", "rvs"])
@pytest.mark.parametrize("weighted", [True, False], ids=["weighted", "unweighted"])
def test_split_bound_scale12(g12, gg12, strategy, weighted):
    """plan.bound = 1 with a dominant return weight (1/p = 4): the extra column is taken
    often; the walks and counters equal the oracle's split-bound walks."""
    lg = oracle.Logic(kind=oracle.NODE2VEC, weighted=weighted, p=0.25, q=2.0)
    pl = oracle.Plan(rho=1.0, bound=1)
    starts = synth.all_vertices(g12["nv"])
    p, ln, st, ora = _run_both(gg12, g12, lg, pl, STRATS[strategy], starts, 20, 77)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)
    if strategy != "rvs":
        assert st["rjs_steps"] > 0


def test_split_bound_fewer_trials_on_gpu(g12, gg12):
    starts = synth.all_vertices(g12["nv"])
    a = gpu_walk(gg12, N2V_RET, oracle.Plan(bound=0), oracle.RJS_ONLY, starts, 20, 5)[2]
    b = gpu_walk(gg12, N2V_RET, oracle.Plan(bound=1), oracle.RJS_ONLY, starts, 20, 5)[2]
    assert b["rjs_trials"] / b["steps"] < 0.75 * a["rjs_trials"] / a["steps"]


@pytest.mark.parametrize("strategy", ["auto", "rjs"])
def test_split_bound_chisquare_hub(strategy):
    g = hub_ring_graph(600)
    gg = GpuGraph(g)
    try:
        assert fw.fw_graph_info(gg.handle)[3]
        _hub_chisq(g, gg, N2V_RET, oracle.Plan(rho=1.0, bound=1), STRATS[strategy], 29, f"split bound {strategy}")
    finally:
        gg.close()


def test_split_bound_needs_symmetric_graph(g12, gg12):
    assert fw.fw_graph_info(gg12.handle)[3]
    dev = torch.device("cuda:0")
    s = torch.zeros(4, dtype=torch.int32, device=dev)
    out = torch.zeros(4 * 6, dtype=torch.int32, device=dev)
    ln = torch.zeros(4, dtype=torch.int32, device=dev)
    # a directed edge 0 -> 1 without its reverse
    gd = synth.csr_from_edges(3, [(0, 1), (0, 2)], h=[1, 2], symmetric=False)
    # reverse edges present but with different h
    gh = synth.csr_from_edges(3, [(0, 1), (1, 2)], h=[1, 2])
    gh["h"] = gh["h"].copy()
    gh["h"][0] += 1.0
    for g in (gd, gh):
        gg = GpuGraph(g)
        try:
            assert not fw.fw_graph_info(gg.handle)[3]
            for split in (fw.fw_plan_default(bound=1), fw.fw_plan_default(bound=2)):
                with pytest.raises(fw.FlexiWalkError) as e:
                    fw.fw_walk(gg.handle, fw.fw_logic_node2vec(0.25, 2.0, True), split, 0, s, 4, 5, 1, out, ln)
                assert e.value.code == fw.FW_E_INVALID
            # second-order PageRank's member board needs no symmetry
            fw.fw_walk(gg.handle, fw.fw_logic_second_pr(0.2, True), fw.fw_plan_default(bound=2), 0, s, 4, 5, 1, out,
                       ln)
            # the paper's bound needs no symmetry
            fw.fw_walk(gg.handle, fw.fw_logic_node2vec(0.25, 2.0, True), fw.fw_plan_default(), 0, s, 4, 5, 1, out,
                       ln)
            torch.cuda.synchronize()
        finally:
            gg.close()
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_walk(gg12.handle, fw.fw_logic_node2vec(0.25, 2.0, True), fw.fw_plan_default(bound=3), 0, s, 4, 5, 1,
                   out, ln)


# ------------------------------------------------------------------ edge index
@pytest.fixture(scope="module")
def gi12(g12):
    gg = GpuGraph(g12, index=True)
    yield gg
    gg.close()


@pytest.mark.parametrize("strategy", list(STRATS), ids=list(STRATS))
@pytest.mark.parametrize("bound", [0, 1, 2])
def test_edge_index_same_walks(g12, gg12, gi12, strategy, bound):
    """The edge index answers u in N(prev) exactly: walks and every counter but the
    algorithmic bytes equal the searched rows'; all counters equal the oracle's with
    indexed byte accounting."""
    lg = oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=0.5, q=2.0)
    pl = oracle.Plan(rho=1.0, bound=bound)
    starts = synth.all_vertices(g12["nv"])
    a = gpu_walk(gg12, lg, pl, STRATS[strategy], starts, 20, 3)
    b = gpu_walk(gi12, lg, pl, STRATS[strategy], starts, 20, 3, lds_cap=16)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    for k in COUNTERS[:-1]:
        assert a[2][k] == b[2][k], k
    ora = oracle.walk(oracle.Graph(g12), lg, oracle.Plan(rho=1.0, bound=bound),
                      STRATS[strategy], starts, 20, 3)
    rep = parity(b[0], b[1], ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(b[2], ora)


@pytest.mark.parametrize("strategy", ["rvs", "auto", "rjs"])
def test_edge_index_hub_rows(strategy):
    """Hub rows of 3000 neighbours with N(prev) never staged: every membership test of
    the eRVS scan goes through the index."""
    g = hub_ring_graph(3000)
    gg = GpuGraph(g, index=True)
    try:
        starts = np.arange(1, 3001, dtype=np.int32)
        pl = oracle.Plan(rho=1.0)
        p, ln, st, ora = _run_both(gg, g, N2V, pl, STRATS[strategy], starts, 6, 11, lds_cap=0)
        rep = parity(p, ln, ora)
        assert_parity(rep)
        if rep["mismatch_walkers"] == 0:
            _assert_counters(st, ora)
    finally:
        gg.close()


def test_edge_index_idempotent_and_tiny_graphs():
    for g in (synth.csr_from_edges(3, [(0, 1)], h=[2]), synth.csr_from_edges(2, [], h=[])):
        gg = GpuGraph(g, index=True)
        try:
            fw.fw_graph_build_index(gg.handle)  # second call is a no-op
            p, ln, st = gpu_walk(gg, N2V, oracle.Plan(), oracle.AUTO, np.zeros(3, np.int32), 4, 1)
            ora = oracle.walk(oracle.Graph(g), N2V, oracle.Plan(), oracle.AUTO,
                              np.zeros(3, np.int32), 4, 1)
            np.testing.assert_array_equal(p, ora.paths)
        finally:
            gg.close()


# ------------------------------------------------------------------ second-order PageRank
PR2 = oracle.Logic(kind=oracle.SECOND_PR, weighted=True, gamma=0.2)


@pytest.mark.parametrize("strategy", list(STRATS), ids=list(STRATS))
@pytest.mark.parametrize("weighted", [True, False], ids=["weighted", "unweighted"])
@pytest.mark.parametrize("indexed", [False, True], ids=["search", "index"])
def test_second_pr_scale12(g12, gg12, gi12, strategy, weighted, indexed):
    """Eq. (2ndpr) with gamma = 0.2, one walker per vertex, L = 20: walks and counters
    equal the oracle's, with the sorted-row search and with the edge index."""
    lg = oracle.Logic(kind=oracle.SECOND_PR, weighted=weighted, gamma=0.2)
    pl = oracle.Plan(rho=1.0)
    starts = synth.all_vertices(g12["nv"])
    gg = gi12 if indexed else gg12
    p, ln, st = gpu_walk(gg, lg, pl, STRATS[strategy], starts, 20, 42)
    ora = oracle.walk(oracle.Graph(g12), lg, pl, STRATS[strategy], starts, 20, 42)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)
    if strategy == "auto":
        assert st["rjs_steps"] > 0 and st["rvs_steps"] > 0


@pytest.mark.parametrize("strategy", list(STRATS), ids=list(STRATS))
def test_second_pr_hub_rows(strategy):
    """Hub rows (eRVS jump scan, N(prev) staged or not) with degrees 2 and 3001 meeting
    in max_d."""
    g = hub_ring_graph(3000)
    gg = GpuGraph(g)
    try:
        starts = np.arange(1, 3001, dtype=np.int32)
        for cap in (2048, 16):
            p, ln, st, ora = _run_both(gg, g, PR2, oracle.Plan(rho=1.0), STRATS[strategy], starts, 6, 13,
                                       lds_cap=cap)
            rep = parity(p, ln, ora)
            assert_parity(rep)
            if rep["mismatch_walkers"] == 0:
                _assert_counters(st, ora)
    finally:
        gg.close()


@pytest.mark.parametrize("strategy", list(STRATS), ids=list(STRATS))
def test_second_pr_chisquare_hub(strategy):
    """Second step at the 600-neighbour hub from leaf 1 against the exact transition."""
    g = hub_ring_graph(600)
    gg = GpuGraph(g)
    try:
        _hub_chisq(g, gg, PR2, oracle.Plan(rho=1.0), STRATS[strategy], 41, f"second-order PageRank {strategy}")
    finally:
        gg.close()


def test_second_pr_logic_errors():
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_logic_second_pr(-0.1)
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_logic_second_pr(float("nan"))
    lg = fw.fw_logic_second_pr(0.3, False)
    assert lg.kind == fw.FW_SECOND_PR and abs(lg.gamma - 0.3) < 1e-7 and lg.weighted == 0


# ------------------------------------------------------------------ comparison selection policies
@pytest.mark.parametrize("strategy", [oracle.RANDOM_SELECT, oracle.DEGREE_SELECT], ids=["random", "degree"])
@pytest.mark.parametrize("logic", [N2V, PR2, MP], ids=["node2vec", "2ndpr", "metapath"])
def test_selection_policies_scale12(g12, gg12, strategy, logic):
    """The fair-coin and degree-threshold policies the paper compares its cost model with:
    walks and counters equal the oracle's."""
    pl = oracle.Plan(rho=1.0, d_lo=24, rjs_cap=256)
    starts = synth.uniform_starts(g12["nv"], 5000, 9)
    p, ln, st, ora = _run_both(gg12, g12, logic, pl, strategy, starts, 20, 77)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)
    assert st["rjs_steps"] > 0 and st["rvs_steps"] > 0


# ------------------------------------------------------------------ skewed property weights
@pytest.mark.parametrize("strategy", list(STRATS), ids=list(STRATS))
@pytest.mark.parametrize("weights", ["pareto1", "pareto3", "degree"])
def test_skewed_weights_scale12(g12, strategy, weights):
    """Power-law (numpy-style Pareto, alpha 1 and 3) and degree-based property weights:
    heavy tails stress the bound, the cost model and the float keys; walks and counters
    equal the oracle's."""
    g = dict(g12)
    if weights == "degree":
        g["h"] = synth.degree_weights(g["row_ptr"], g["col"])
    else:
        g["h"] = synth.pareto_weights(g["row_ptr"], g["col"], float(weights[6:]), 7)
    gg = GpuGraph(g)
    try:
        assert fw.fw_graph_info(gg.handle)[3] == (weights != "degree")
        pl = oracle.Plan(rho=1.0, rjs_cap=256)
        starts = synth.all_vertices(g["nv"])
        p, ln, st, ora = _run_both(gg, g, N2V, pl, STRATS[strategy], starts, 15, 5)
        rep = parity(p, ln, ora)
        assert_parity(rep)
        if rep["mismatch_walkers"] == 0:
            _assert_counters(st, ora)
    finally:
        gg.close()


# ------------------------------------------------------------------ h-proportional proposals
@pytest.fixture(scope="module")
def ga12(g12):
    gg = GpuGraph(g12, index=True, alias=True)
    yield gg
    gg.close()


HP_LOGICS = {"n2v": N2V, "n2v_ret": N2V_RET, "2ndpr": PR2, "metapath": MP,
             "n2v_unweighted": oracle.Logic(kind=oracle.NODE2VEC, weighted=False, p=0.25, q=2.0)}


@pytest.mark.parametrize("strategy", ["auto", "rjs"])
@pytest.mark.parametrize("bound", [0, 1, 2])
@pytest.mark.parametrize("logic", list(HP_LOGICS), ids=list(HP_LOGICS))
def test_h_proposals_scale12(g12, ga12, strategy, bound, logic):
    """plan.proposal = 1: alias-table proposals, the test on w; walks and counters equal
    the oracle's (which builds its alias tables independently)."""
    lg = HP_LOGICS[logic]
    pl = oracle.Plan(rho=1.0, bound=bound if lg.kind != oracle.METAPATH else 0, proposal=1, rjs_cap=256)
    starts = synth.all_vertices(g12["nv"])
    p, ln, st, ora = _run_both(ga12, g12, lg, pl, STRATS[strategy], starts, 20, 31)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)
    assert st["rjs_steps"] > 0


@pytest.mark.parametrize("weights", ["pareto1", "pareto2"])
def test_h_proposals_skewed(g12, weights):
    """Heavy-tailed weights, where uniform proposals need hundreds of trials per step."""
    g = dict(g12)
    g["h"] = synth.pareto_weights(g["row_ptr"], g["col"], float(weights[6:]), 7)
    gg = GpuGraph(g, alias=True)
    try:
        starts = synth.all_vertices(g["nv"])
        for prop in (0, 1):
            pl = oracle.Plan(rho=1.0, proposal=prop, rjs_cap=4096)
            p, ln, st, ora = _run_both(gg, g, N2V, pl, oracle.RJS_ONLY, starts, 12, 19)
            rep = parity(p, ln, ora)
            assert_parity(rep)
            if rep["mismatch_walkers"] == 0:
                _assert_counters(st, ora)
            if prop == 0:
                uniform_trials = st["rjs_trials"]
        assert st["rjs_trials"] < 0.1 * uniform_trials
    finally:
        gg.close()


def test_h_proposals_chisquare_hub():
    g = hub_ring_graph(600)
    gg = GpuGraph(g, alias=True)
    try:
        _hub_chisq(g, gg, N2V_RET, oracle.Plan(rho=1.0, bound=1, proposal=1), oracle.RJS_ONLY, 43, "h proposals")
    finally:
        gg.close()


def test_h_proposals_need_alias(g12, gg12):
    dev = torch.device("cuda:0")
    s = torch.zeros(4, dtype=torch.int32, device=dev)
    out = torch.zeros(4 * 6, dtype=torch.int32, device=dev)
    ln = torch.zeros(4, dtype=torch.int32, device=dev)
    with pytest.raises(fw.FlexiWalkError) as e:
        fw.fw_walk(gg12.handle, fw.fw_logic_node2vec(0.5, 2.0, True), fw.fw_plan_default(proposal=1), 0, s, 4, 5, 1,
                   out, ln)
    assert e.value.code == fw.FW_E_STATE
    # unweighted logics ignore it
    fw.fw_walk(gg12.handle, fw.fw_logic_node2vec(0.5, 2.0, False), fw.fw_plan_default(proposal=1), 0, s, 4, 5, 1,
               out, ln)
    torch.cuda.synchronize()


# ------------------------------------------------------------------ member board (plan.bound = 2)
@pytest.fixture(scope="module")
def gn12(g12):
    gg = GpuGraph(g12, alias=True)  # alias records without the edge index
    yield gg
    gg.close()


MB_LOGICS = {"n2v_q2": oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=0.5, q=2.0), "n2v_ret": N2V_RET,
             "n2v_q05": N2V, "2ndpr": PR2, "2ndpr_g07": oracle.Logic(kind=oracle.SECOND_PR, weighted=True, gamma=0.7),
             "n2v_unweighted": oracle.Logic(kind=oracle.NODE2VEC, weighted=False, p=0.25, q=4.0),
             "2ndpr_unweighted": oracle.Logic(kind=oracle.SECOND_PR, weighted=False, gamma=0.2)}


@pytest.mark.parametrize("strategy", ["auto", "rjs"])
@pytest.mark.parametrize("proposal", [0, 1], ids=["uniform", "hprop"])
@pytest.mark.parametrize("indexed", [False, True], ids=["search", "index"])
@pytest.mark.parametrize("logic", list(MB_LOGICS), ids=list(MB_LOGICS))
def test_member_board_scale12(g12, gn12, ga12, strategy, proposal, indexed, logic):
    """plan.bound = 2: per step the smaller of the member board and the split (Node2Vec)
    or plain board; a member-region trial finds (cur, x) and its h through the edge index
    or a search of cur's row.  Walks and counters equal the oracle's."""
    lg = MB_LOGICS[logic]
    pl = oracle.Plan(rho=1.0, bound=2, proposal=proposal, rjs_cap=256)
    starts = synth.all_vertices(g12["nv"])
    p, ln, st, ora = _run_both(ga12 if indexed else gn12, g12, lg, pl, STRATS[strategy], starts, 20, 53)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)
    assert st["rjs_steps"] > 0


def test_member_board_fewer_trials_on_gpu(g12, ga12):
    """Second-order PageRank: the plain bound is loose where d(v) >> d(v'); the member
    board's area does not grow with d(v) / d(v')."""
    starts = synth.all_vertices(g12["nv"])
    for prop in (0, 1):
        a = gpu_walk(ga12, PR2, oracle.Plan(bound=0, proposal=prop), oracle.RJS_ONLY, starts, 20, 5)[2]
        b = gpu_walk(ga12, PR2, oracle.Plan(bound=2, proposal=prop), oracle.RJS_ONLY, starts, 20, 5)[2]
        assert b["rjs_trials"] / b["steps"] < 0.5 * a["rjs_trials"] / a["steps"], prop


@pytest.mark.parametrize("logic", ["n2v_ret", "2ndpr"])
@pytest.mark.parametrize("proposal", [0, 1], ids=["uniform", "hprop"])
def test_member_board_chisquare_hub(logic, proposal):
    """Second step at the 600-neighbour hub from leaf 1 (two members, the ring neighbours
    of leaf 1) against the exact transition."""
    lg = MB_LOGICS[logic]
    g = hub_ring_graph(600)
    gg = GpuGraph(g, index=True, alias=True)
    try:
        _hub_chisq(g, gg, lg, oracle.Plan(rho=1.0, bound=2, proposal=proposal), oracle.RJS_ONLY, 47,
                   f"member board {logic} {proposal}")
    finally:
        gg.close()


# ------------------------------------------------------------------ 8-bit property weights
def _q8(g):
    codes, scale = synth.quantize_u8(g["h"])
    gq = dict(g, h=None, h8=codes, h_scale=scale)
    gf = dict(g, h=(codes.astype(np.float64) * np.float64(scale)).astype(np.float32))
    return gq, gf


Q8_LOGICS = {"n2v": oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=0.5, q=2.0), "2ndpr": PR2, "metapath": MP}


@pytest.mark.parametrize("strategy", list(STRATS), ids=list(STRATS))
@pytest.mark.parametrize("logic", list(Q8_LOGICS), ids=list(Q8_LOGICS))
@pytest.mark.parametrize("plan", ["paper", "member_h"])
def test_h8_scale12(g12, strategy, logic, plan):
    """8-bit weights (4-byte edge records): walks and counters equal the oracle's on the
    same codes, and walks equal the GPU's own walks on the float graph of the dequantised
    weights (whose byte counter moves 3 bytes more per scanned or proposed edge)."""
    gq, gf = _q8(g12)
    lg = Q8_LOGICS[logic]
    pl = (oracle.Plan(rho=1.0) if plan == "paper" else
          oracle.Plan(rho=1.0, bound=2 if lg.kind != oracle.METAPATH else 0, proposal=1))
    ggq = GpuGraph(gq, index=plan != "paper", alias=plan != "paper")
    ggf = GpuGraph(gf, index=plan != "paper", alias=plan != "paper")
    try:
        starts = synth.all_vertices(g12["nv"])
        p, ln, st = gpu_walk(ggq, lg, pl, STRATS[strategy], starts, 20, 61)
        pf, lf, stf = gpu_walk(ggf, lg, pl, STRATS[strategy], starts, 20, 61)
    finally:
        ggq.close()
        ggf.close()
    np.testing.assert_array_equal(p, pf)
    np.testing.assert_array_equal(ln, lf)
    assert st["alg_bytes"] < stf["alg_bytes"]
    ora = oracle.walk(oracle.Graph(gq), lg, pl, STRATS[strategy], starts, 20, 61)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)


def test_h8_wide_graph(g12):
    """More than 2^24 vertices: the 8-bit weights fall back to 8-byte records of the
    dequantised weight; walks and counters still equal the oracle's."""
    gq, _ = _q8(g12)
    nv = (1 << 24) + 64
    rp = np.full(nv + 1, g12["ne"], np.int64)
    rp[: g12["nv"] + 1] = g12["row_ptr"]
    gw = dict(gq, nv=nv, row_ptr=rp, label=None)
    gg = GpuGraph(gw)
    try:
        starts = synth.all_vertices(g12["nv"])
        p, ln, st, ora = _run_both(gg, gw, N2V, oracle.Plan(rho=1.0), oracle.AUTO, starts, 12, 67)
    finally:
        gg.close()
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)


def test_h8_argument_errors(g12):
    gq, _ = _q8(g12)
    for bad in (dict(gq, h_scale=0.0), dict(gq, h_scale=float("inf")), dict(gq, h=g12["h"])):
        with pytest.raises(fw.FlexiWalkError) as e:
            GpuGraph(bad)
        assert e.value.code == fw.FW_E_INVALID


def _alias_graphs():
    out = {}
    g = synth.rmat(12, 8 << 12, seed=1, nlabels=5)
    out["rmat12"] = g
    out["unweighted"] = dict(g, h=None)
    gz = synth.rmat(11, 8 << 11, seed=4)
    hz = gz["h"].copy()
    hz[::3] = 0.0  # zero weights, and rows whose weights are all zero
    gz["h"] = hz
    out["zeros"] = gz
    gp = synth.rmat(12, 8 << 12, seed=3)
    gp["h"] = synth.pareto_weights(gp["row_ptr"], gp["col"], 1.0, 5)
    out["pareto1"] = gp
    out["hub600"] = hub_ring_graph(600)
    # one row of 200,000 entries (many 64-entry tiles of the scan and of both merges)
    n = 200000
    star = synth.csr_from_edges(n + 1, [(0, i) for i in range(1, n + 1)])
    star["h"] = synth.pareto_weights(star["row_ptr"], star["col"], 1.5, 9)
    out["star200k"] = star
    return out


@pytest.mark.parametrize("name", ["rmat12", "unweighted", "zeros", "pareto1", "hub600", "star200k"])
def test_alias_tables_equal_oracle(name):
    """The proposal records' alias tables (built on the GPU, one wave per row, by prefix
    sums and merges) equal the oracle's sequential sweep entry for entry."""
    g = _alias_graphs()[name]
    gg = GpuGraph(g, alias=True)
    try:
        thr, al = fw.fw_graph_export_alias(gg.handle, gg.ne)
    finally:
        gg.close()
    othr, oal = oracle.Graph(g).alias()
    np.testing.assert_array_equal(al, oal)
    np.testing.assert_array_equal(thr, othr)


def test_alias_build_runs_preprocessing(g12):
    """fw_graph_build_alias on a graph not yet preprocessed preprocesses it first (its
    records carry the candidates' vertex records, h_MAX and h_SUM included): walks with
    h-proportional proposals then equal the oracle's."""
    gg = GpuGraph(g12, preprocess=False)
    try:
        fw.fw_graph_build_alias(gg.handle)
        torch.cuda.synchronize()
        hmax, hsum = fw.fw_graph_export_aux(gg.handle, gg.nv)
        ohmax, ohsum = oracle.Graph(g12).aux()
        np.testing.assert_array_equal(hmax, ohmax)
        np.testing.assert_array_equal(hsum, ohsum)
        pl = oracle.Plan(rho=1.0, proposal=1, bound=2)
        starts = synth.all_vertices(g12["nv"])
        p, ln, st, ora = _run_both(gg, g12, N2V_RET, pl, oracle.AUTO, starts, 12, 83)
        rep = parity(p, ln, ora)
        assert_parity(rep)
        if rep["mismatch_walkers"] == 0:
            _assert_counters(st, ora)
    finally:
        gg.close()
