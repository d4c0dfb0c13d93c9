"""Batched launches: many queries with their own p, q (or schema), L, seed and starts in
one persistent launch, optionally captured into a HIP graph (needs an MI355X).

Each query must equal the same query run alone with fw_walk (bit for bit) and the
oracle's walks from the query's seed (to the parity bar); graph replays must equal the
eager launch on every replay.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import GpuGraph, assert_parity, fw_plan, gpu_walk, parity

import paper_2512_00705_amd as fw

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def g12():
    return synth.rmat(12, 8 << 12, seed=1, nlabels=5)


@pytest.fixture(scope="module")
def gg12(g12):
    gg = GpuGraph(g12)
    yield gg
    gg.close()


def _queries(qd, logics):
    out = []
    for i, lg in enumerate(logics):
        q = fw.fw_query()
        q.logic = lg
        q.n, q.L, q.seed = int(qd["n"][i]), int(qd["L"][i]), int(qd["seed"][i])
        q.start_off, q.out_off, q.len_off = int(qd["start_off"][i]), int(qd["out_off"][i]), int(qd["len_off"][i])
        out.append(q)
    return out


class Batch:
    def __init__(self, gg, qd, logics, plan, strategy):
        self.qd = qd
        n = qd["n"].astype(np.int64)
        # buffers sized from the offsets the queries address, never from a recount
        need_starts = int((qd["start_off"] + n).max(initial=0))
        need_paths = int((qd["out_off"] + n * (qd["L"].astype(np.int64) + 1)).max(initial=0))
        need_len = int((qd["len_off"] + n).max(initial=0))
        assert qd["starts"].shape[0] >= need_starts
        self.starts = torch.from_numpy(qd["starts"]).to(DEV)
        self.paths = torch.full((max(need_paths, 1),), -7, dtype=torch.int32, device=DEV)
        self.lengths = torch.full((max(need_len, 1),), -7, dtype=torch.int32, device=DEV)
        self.stats = torch.zeros(fw.FW_NSTATS, dtype=torch.int64, device=DEV)
        self.h = fw.fw_batch_create(gg.handle, _queries(qd, logics), plan, strategy, self.starts, self.paths,
                                    self.lengths)

    def query(self, i):
        n, L = int(self.qd["n"][i]), int(self.qd["L"][i])
        o, lo = int(self.qd["out_off"][i]), int(self.qd["len_off"][i])
        p = self.paths[o:o + n * (L + 1)].view(n, L + 1).cpu().numpy() if n else np.zeros((0, L + 1), np.int32)
        return p, self.lengths[lo:lo + n].cpu().numpy()

    def close(self):
        torch.cuda.synchronize()
        fw.fw_batch_destroy(self.h)


def _small_batch(nv, nq, seed):
    return synth.batch_queries(nv, nq, seed, n_max=400, L_lo=0, L_hi=25)


@pytest.mark.parametrize("strategy", [oracle.AUTO, oracle.RVS_ONLY, oracle.RJS_ONLY], ids=["auto", "rvs", "rjs"])
def test_batch_equals_alone_and_oracle(g12, gg12, strategy):
    qd = _small_batch(g12["nv"], 40, 3)
    qd["n"][5] = 0  # an empty query
    logics = [oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=float(qd["p"][i]), q=float(qd["q"][i]))
              for i in range(40)]
    pl = oracle.Plan(rho=4.0)
    b = Batch(gg12, qd, [fw.fw_logic_node2vec(l.p, l.q, True) for l in logics], fw_plan(pl), strategy)
    try:
        fw.fw_batch_launch(b.h, b.stats)
        fw.fw_graph_check(gg12.handle)
        og = oracle.Graph(g12)
        total_steps = 0
        for i in range(40):
            n = int(qd["n"][i])
            p, ln = b.query(i)
            st = qd["starts"][qd["start_off"][i]:qd["start_off"][i] + n]
            if n == 0:
                continue
            alone = gpu_walk(gg12, logics[i], pl, strategy, st, int(qd["L"][i]), int(qd["seed"][i]))
            np.testing.assert_array_equal(p, alone[0])
            np.testing.assert_array_equal(ln, alone[1])
            ora = oracle.walk(og, logics[i], pl, strategy, st, int(qd["L"][i]), int(qd["seed"][i]))
            assert_parity(parity(p, ln, ora))
            total_steps += int(ln.sum())
        assert int(b.stats[0].item()) == total_steps
    finally:
        b.close()


def test_batch_metapath(g12, gg12):
    qd = _small_batch(g12["nv"], 16, 8)
    schemas = [tuple(int(x) for x in np.random.default_rng(i).integers(0, 5, 1 + i % 6)) for i in range(16)]
    logics = [oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=s) for s in schemas]
    pl = oracle.Plan(rho=2.0, rjs_cap=32)
    b = Batch(gg12, qd, [fw.fw_logic_metapath(list(s), True) for s in schemas], fw_plan(pl), oracle.AUTO)
    try:
        fw.fw_batch_launch(b.h)
        og = oracle.Graph(g12)
        for i in range(16):
            n = int(qd["n"][i])
            p, ln = b.query(i)
            st = qd["starts"][qd["start_off"][i]:qd["start_off"][i] + n]
            ora = oracle.walk(og, logics[i], pl, oracle.AUTO, st, int(qd["L"][i]), int(qd["seed"][i]))
            assert_parity(parity(p, ln, ora))
    finally:
        b.close()


def test_batch_graph_replay(g12, gg12):
    """Captured once, replayed three times with eager work in between; every replay
    writes exactly the eager result."""
    qd = _small_batch(g12["nv"], 64, 21)
    lgs = [fw.fw_logic_node2vec(float(qd["p"][i]), float(qd["q"][i]), True) for i in range(64)]
    b = Batch(gg12, qd, lgs, fw.fw_plan_default(rho=4.0), fw.FW_AUTO)
    stream = torch.cuda.Stream()
    try:
        fw.fw_batch_launch(b.h)
        torch.cuda.synchronize()
        ref_p, ref_l = b.paths.clone(), b.lengths.clone()
        with torch.cuda.stream(stream):
            fw.fw_batch_capture(b.h, b.stats, stream)
        for rep in range(3):
            b.paths.fill_(-9)
            b.lengths.fill_(-9)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                fw.fw_batch_replay(b.h, stream)
            stream.synchronize()
            assert torch.equal(b.paths, ref_p), rep
            assert torch.equal(b.lengths, ref_l), rep
            # eager work between replays
            gpu_walk(gg12, oracle.Logic(kind=oracle.NODE2VEC, p=1.0, q=1.0), oracle.Plan(), oracle.AUTO,
                     np.arange(100, dtype=np.int32), 5, rep)
        assert int(b.stats[0].item()) == 3 * int(ref_l.sum().item())
    finally:
        b.close()


def test_batch_argument_errors(g12, gg12):
    qd = _small_batch(g12["nv"], 2, 1)
    lgs = [fw.fw_logic_node2vec(1.0, 1.0, True), fw.fw_logic_metapath([0, 1], True)]
    dev = torch.zeros(16, dtype=torch.int32, device=DEV)
    with pytest.raises(fw.FlexiWalkError):  # mixed kinds
        fw.fw_batch_create(gg12.handle, _queries(qd, lgs), fw.fw_plan_default(), 0, dev, dev, dev)
    q = _queries(qd, [lgs[0]])
    q[0].L = -1
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_batch_create(gg12.handle, q, fw.fw_plan_default(), 0, dev, dev, dev)
    q = _queries(qd, [lgs[0]])
    q[0].n = 17  # block larger than the 16-element arrays
    q[0].start_off = q[0].out_off = q[0].len_off = 0
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_batch_create(gg12.handle, q, fw.fw_plan_default(), 0, dev, dev, dev)
    empty = fw.fw_batch_create(gg12.handle, [], fw.fw_plan_default(), 0, None, None, None)
    fw.fw_batch_launch(empty)
    fw.fw_batch_destroy(empty)


@pytest.mark.parametrize("bound", [1, 2], ids=["split", "member"])
def test_batch_split_bound(g12, gg12, bound):
    qd = _small_batch(g12["nv"], 24, 13)
    logics = [oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=float(0.25 + (i % 4) * 0.5), q=2.0)
              for i in range(24)]
    pl = oracle.Plan(rho=1.0, bound=bound)
    b = Batch(gg12, qd, [fw.fw_logic_node2vec(l.p, l.q, True) for l in logics], fw_plan(pl), oracle.AUTO)
    try:
        fw.fw_batch_launch(b.h)
        og = oracle.Graph(g12)
        for i in range(24):
            n = int(qd["n"][i])
            if n == 0:
                continue
            p, ln = b.query(i)
            st = qd["starts"][qd["start_off"][i]:qd["start_off"][i] + n]
            alone = gpu_walk(gg12, logics[i], pl, oracle.AUTO, st, int(qd["L"][i]), int(qd["seed"][i]))
            np.testing.assert_array_equal(p, alone[0])
            ora = oracle.walk(og, logics[i], pl, oracle.AUTO, st, int(qd["L"][i]), int(qd["seed"][i]))
            assert_parity(parity(p, ln, ora))
    finally:
        b.close()


@pytest.mark.parametrize("bound", [0, 2], ids=["paper", "member"])
def test_batch_second_pr(g12, gg12, bound):
    """A batch of second-order PageRank queries with their own gamma, L, seed and starts."""
    qd = _small_batch(g12["nv"], 20, 17)
    gammas = [0.05 * (i % 20) for i in range(20)]
    logics = [oracle.Logic(kind=oracle.SECOND_PR, weighted=True, gamma=g) for g in gammas]
    pl = oracle.Plan(rho=1.0, bound=bound)
    b = Batch(gg12, qd, [fw.fw_logic_second_pr(l.gamma, True) for l in logics], fw_plan(pl), oracle.AUTO)
    try:
        fw.fw_batch_launch(b.h)
        og = oracle.Graph(g12)
        for i in range(20):
            n = int(qd["n"][i])
            if n == 0:
                continue
            p, ln = b.query(i)
            st = qd["starts"][qd["start_off"][i]:qd["start_off"][i] + n]
            alone = gpu_walk(gg12, logics[i], pl, oracle.AUTO, st, int(qd["L"][i]), int(qd["seed"][i]))
            np.testing.assert_array_equal(p, alone[0])
            ora = oracle.walk(og, logics[i], pl, oracle.AUTO, st, int(qd["L"][i]), int(qd["seed"][i]))
            assert_parity(parity(p, ln, ora))
    finally:
        b.close()


def test_autotune_mix(g12, gg12):
    """One plan for a mix of logics: valid fields, bounds every logic accepts, and a batch
    run with it equals the oracle."""
    logics = [fw.fw_logic_node2vec(0.5, 2.0, True), fw.fw_logic_node2vec(2.0, 0.5, True),
              fw.fw_logic_second_pr(0.2, True)]
    pl = fw.fw_plan_autotune_mix(gg12.handle, logics)
    assert pl.rho > 0 and pl.bound in (0, 1, 2) and pl.proposal == 0 and pl.grid >= 0 and pl.lanes == 64
    assert pl.hub_deg == 0 and pl.hub_lanes == 64  # a mix keeps P = 64 (batches and servers run no hub lanes)
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_plan_autotune_mix(gg12.handle, [])
    # Node2Vec on a graph without equal reverse edges: only the paper's bound is tried
    # each vertex points to its successor and to the one 3 ahead (no reverse edges, no duplicates)
    gd = synth.csr_from_edges(64, [(i, (i + 1) % 64) for i in range(64)] + [(i, (i + 3) % 64) for i in range(64)],
                              h=[1 + (i % 5) for i in range(128)], symmetric=False)
    gg = GpuGraph(gd)
    try:
        assert not fw.fw_graph_info(gg.handle)[3]
        pd = fw.fw_plan_autotune_mix(gg.handle, [fw.fw_logic_node2vec(0.25, 2.0, True),
                                                 fw.fw_logic_second_pr(0.3, True)])
        assert pd.bound == 0
    finally:
        gg.close()
    # a mix one batch can hold (the two Node2Vec logics) is tuned by timing such a batch;
    # that plan drives a batch of them exactly as the oracle walks them
    pl = fw.fw_plan_autotune_mix(gg12.handle, logics[:2])
    assert pl.rho > 0 and pl.bound in (0, 1, 2) and pl.proposal == 0 and pl.grid >= 0
    qd = _small_batch(g12["nv"], 9, 23)
    olg = [oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=0.5, q=2.0),
           oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=2.0, q=0.5)]
    opl = oracle.Plan(rho=pl.rho, d_lo=pl.d_lo, rjs_cap=pl.rjs_cap, bound=pl.bound, proposal=pl.proposal)
    b = Batch(gg12, qd, [logics[i % 2] for i in range(9)], pl, oracle.AUTO)
    try:
        fw.fw_batch_launch(b.h)
        og = oracle.Graph(g12)
        for i in range(9):
            n = int(qd["n"][i])
            if n == 0:
                continue
            p, ln = b.query(i)
            st = qd["starts"][qd["start_off"][i]:qd["start_off"][i] + n]
            ora = oracle.walk(og, olg[i % 2], opl, oracle.AUTO, st, int(qd["L"][i]), int(qd["seed"][i]))
            assert_parity(parity(p, ln, ora))
    finally:
        b.close()

