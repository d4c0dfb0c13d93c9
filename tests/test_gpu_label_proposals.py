"""Label-conditioned MetaPath proposals on the GPU (needs an MI355X).

plan.proposal = 2: a MetaPath step proposes from the wanted label's group of the row
through that group's alias table (fw_graph_build_label_alias), so one trial samples the
step.  The oracle builds the same groups and tables from their definition and replays
the walks; the bar is the one of the other parity tests (identical walks up to flagged
1e-6 margins, equal counters when nothing differs) and a chi-square at a hub against the
exact transition.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import exact
from tests._gpu import GpuGraph, assert_parity, fw_logic, gpu_walk, parity
from tests._helpers import assert_chisq, chisq_pvalue, triangle_graph
from tests.test_gpu_parity import COUNTERS, STRATS, _assert_counters

import paper_2512_00705_amd as fw

pytestmark = pytest.mark.gpu

MP = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2, 3, 4))
MP_U = oracle.Logic(kind=oracle.METAPATH, weighted=False, schema=(3, 1, 4, 1))
ALL_STRATS = dict(STRATS, random=oracle.RANDOM_SELECT, degree=oracle.DEGREE_SELECT)


@pytest.fixture(scope="module")
def g12():
    return synth.rmat(12, 8 << 12, seed=1, nlabels=5)


@pytest.fixture(scope="module")
def gl12(g12):
    gg = GpuGraph(g12, label_alias=True)
    yield gg
    gg.close()


@pytest.mark.parametrize("strategy", list(ALL_STRATS), ids=list(ALL_STRATS))
@pytest.mark.parametrize("logic", ["weighted", "unweighted"])
def test_label_proposals_scale12(g12, gl12, strategy, logic):
    """R-MAT scale 12 with labels 0..4, 5000 uniform starts, L = 20: every strategy, rho 4
    (rows of degree <= 4 go to eRVS under AUTO), d_lo 16 for the degree policy."""
    lg = MP if logic == "weighted" else MP_U
    pl = oracle.Plan(rho=4.0, d_lo=16 if strategy == "degree" else 0, proposal=2)
    starts = synth.uniform_starts(g12["nv"], 5000, 42)
    p, ln, st = gpu_walk(gl12, lg, pl, ALL_STRATS[strategy], starts, 20, 42)
    ora = oracle.walk(oracle.Graph(g12), lg, pl, ALL_STRATS[strategy], starts, 20, 42)
    rep = parity(p, ln, ora)
    assert_parity(rep)
    if rep["mismatch_walkers"] == 0:
        _assert_counters(st, ora)
    if strategy in ("rjs", "auto"):
        assert st["rjs_steps"] > 0 and st["rjs_trials"] == st["rjs_steps"]
    assert st["ended_early"] > 0


def test_label_proposals_chisquare():
    """Second step from a hub whose 600 neighbours carry labels 0..4 (hashed weights):
    the step's label-1 group against the exact transition."""
    n_leaves = 600
    edges = [(0, i) for i in range(1, n_leaves + 1)] + [(i, i % n_leaves + 1) for i in range(1, n_leaves + 1)]
    lab = [i % 5 for i in range(1, n_leaves + 1)] + [0] * n_leaves
    g = synth.csr_from_edges(n_leaves + 1, edges, label=lab)
    g["h"], _ = synth.edge_props(g["row_ptr"], g["col"], 9)
    lg = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(1, 1))
    gg = GpuGraph(g, label_alias=True)
    try:
        n = 300000

        def pvalue(sd):
            p, ln, st = gpu_walk(gg, lg, oracle.Plan(proposal=2), oracle.RJS_ONLY, np.zeros(n, np.int32), 1, sd)
            counts = {int(v): int(c) for v, c in zip(*np.unique(p[:, 1], return_counts=True))}
            return chisq_pvalue(counts, exact.transition(g, lg, 0, -1, 0), n)
        assert_chisq(pvalue, 37, "label groups at the hub")
    finally:
        gg.close()


def test_label_proposals_errors_and_zero_group(g12):
    lg = fw.fw_logic_metapath([0, 1], True)
    dev = torch.device("cuda:0")
    s = torch.zeros(4, dtype=torch.int32, device=dev)
    out = torch.zeros(4 * 6, dtype=torch.int32, device=dev)
    ln = torch.zeros(4, dtype=torch.int32, device=dev)
    gg = GpuGraph(g12)  # no label groups built
    try:
        with pytest.raises(fw.FlexiWalkError):
            fw.fw_walk(gg.handle, lg, fw.fw_plan_default(proposal=2), 0, s, 4, 5, 1, out, ln)
        with pytest.raises(fw.FlexiWalkError):
            fw.fw_walk(gg.handle, lg, fw.fw_plan_default(proposal=3), 0, s, 4, 5, 1, out, ln)
    finally:
        gg.close()
    # no labels at all
    gn = GpuGraph(synth.rmat(6, 64, seed=1))
    try:
        with pytest.raises(fw.FlexiWalkError):
            fw.fw_graph_build_label_alias(gn.handle)
    finally:
        gn.close()
    # a label of 16 or more
    g16 = synth.csr_from_edges(3, [(0, 1), (1, 2)], h=[1.0, 2.0], label=[16, 0])
    gb = GpuGraph(g16)
    try:
        with pytest.raises(fw.FlexiWalkError):
            fw.fw_graph_build_label_alias(gb.handle)
    finally:
        gb.close()
    # a group whose weights are all 0 ends the walk, as in the oracle
    gz = synth.csr_from_edges(4, [(0, 1), (0, 2), (0, 3)], h=[0.0, 0.0, 5.0], label=[0, 0, 1])
    gzz = GpuGraph(gz, label_alias=True)
    try:
        for schema in ((0, 1), (1, 0)):
            lz = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=schema)
            st = np.zeros(64, np.int32)
            p, ln2, _ = gpu_walk(gzz, lz, oracle.Plan(proposal=2), oracle.RJS_ONLY, st, 3, 4)
            ora = oracle.walk(oracle.Graph(gz), lz, oracle.Plan(proposal=2), oracle.RJS_ONLY, st, 3, 4)
            np.testing.assert_array_equal(p, ora.paths)
            np.testing.assert_array_equal(ln2, ora.lengths)
    finally:
        gzz.close()


def test_label_proposals_batch_and_autotune(g12, gl12):
    """A batch of MetaPath queries with label-conditioned proposals walks as the oracle;
    the autotuner offers the label proposals for a MetaPath logic once the groups exist."""
    from tests._gpu import fw_plan
    from tests.test_gpu_batch import Batch, _small_batch
    qd = _small_batch(g12["nv"], 12, 19)
    lgs = [MP, MP_U, oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(2, 4))]
    # a batch holds one weighting: the weighted logics here, the unweighted one alone
    for group in ([lgs[0], lgs[2]], [lgs[1]]):
        logics = [group[i % len(group)] for i in range(12)]
        pl = oracle.Plan(rho=2.0, proposal=2)
        b = Batch(gl12, qd, [fw_logic(l) for l in logics], fw_plan(pl), oracle.AUTO)
        try:
            fw.fw_batch_launch(b.h, b.stats)
            og = oracle.Graph(g12)
            for i in range(12):
                n = int(qd["n"][i])
                if n == 0:
                    continue
                p, ln = b.query(i)
                st = qd["starts"][qd["start_off"][i]:qd["start_off"][i] + n]
                ora = oracle.walk(og, logics[i], pl, oracle.AUTO, st, int(qd["L"][i]), int(qd["seed"][i]))
                assert_parity(parity(p, ln, ora))
        finally:
            b.close()
    tuned = fw.fw_plan_autotune(gl12.handle, fw_logic(MP))
    assert tuned.proposal in (0, 2)
