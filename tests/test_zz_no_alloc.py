"""The allocation-free batch entry point (needs an MI355X).

fw_batch_run_noalloc keeps its query table and walker counter in a library-owned static
device array; its walks must equal those of fw_batch_create + fw_batch_launch on the same
queries, bit for bit, on consecutive calls that reuse the array with a smaller batch.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import GpuGraph, fw_plan
from tests.test_gpu_batch import Batch, _queries

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


def _noalloc(gg, qd, logics, plan, strategy, b):
    """Runs the batch through fw_batch_run_noalloc into fresh buffers shaped like b's."""
    paths = torch.full_like(b.paths, -7)
    lengths = torch.full_like(b.lengths, -7)
    stats = torch.zeros(fw.FW_NSTATS, dtype=torch.int64, device=DEV)
    fw.fw_batch_run_noalloc(gg.handle, _queries(qd, logics), plan, strategy, b.starts, paths, lengths, stats)
    fw.fw_graph_check(gg.handle)
    torch.cuda.synchronize()
    return paths, lengths, stats


def test_noalloc_equals_batch_twice(g12, gg12):
    # first call: 40 Node2Vec queries; second call: a smaller MetaPath batch that reuses
    # (and must fully overwrite) the table of the first
    qa = synth.batch_queries(g12["nv"], 40, 3, n_max=400, L_lo=0, L_hi=25)
    qa["n"][5] = 0
    la = [fw.fw_logic_node2vec(float(qa["p"][i]), float(qa["q"][i]), True) for i in range(40)]
    qb = synth.batch_queries(g12["nv"], 9, 11, n_max=100, L_lo=1, L_hi=12)
    lb = [fw.fw_logic_metapath([int(x) for x in np.random.default_rng(i).integers(0, 5, 1 + i % 4)], True)
          for i in range(9)]
    plan = fw_plan(oracle.Plan(rho=4.0, rjs_cap=64))
    for qd, logics in ((qa, la), (qb, lb)):
        b = Batch(gg12, qd, logics, plan, fw.FW_AUTO)
        try:
            fw.fw_batch_launch(b.h, b.stats)
            torch.cuda.synchronize()
            p, ln, st = _noalloc(gg12, qd, logics, plan, fw.FW_AUTO, b)
            assert torch.equal(p, b.paths)
            assert torch.equal(ln, b.lengths)
            assert torch.equal(st, b.stats)
            assert int(st[0].item()) > 0
        finally:
            b.close()


def test_noalloc_limits(g12, gg12):
    qd = synth.batch_queries(g12["nv"], 4, 5, n_max=8, L_lo=1, L_hi=4)
    lg = [fw.fw_logic_node2vec(1.0, 1.0, True)] * 4
    b = Batch(gg12, qd, lg, fw.fw_plan_default(), fw.FW_AUTO)
    try:
        too_many = _queries(qd, lg)[:1] * (fw.FW_NOALLOC_MAX_QUERIES + 1)
        for q in too_many:
            q.n = 0
        with pytest.raises(fw.FlexiWalkError) as e:
            fw.fw_batch_run_noalloc(gg12.handle, too_many, fw.fw_plan_default(), fw.FW_AUTO, b.starts, b.paths,
                                    b.lengths)
        assert e.value.code == fw.FW_E_INVALID
        # a query whose block leaves the caller's arrays is refused before anything runs
        bad = _queries(qd, lg)
        bad[0].out_off = int(b.paths.numel())
        with pytest.raises(fw.FlexiWalkError) as e:
            fw.fw_batch_run_noalloc(gg12.handle, bad, fw.fw_plan_default(), fw.FW_AUTO, b.starts, b.paths, b.lengths)
        assert e.value.code == fw.FW_E_INVALID
        # an empty batch is a no-op
        fw.fw_batch_run_noalloc(gg12.handle, [], fw.fw_plan_default(), fw.FW_AUTO, b.starts, b.paths, b.lengths)
    finally:
        b.close()
