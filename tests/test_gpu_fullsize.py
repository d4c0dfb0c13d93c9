"""Full-size workloads on the GPU, checked on sampled walkers and by invariants.

Scale-22 R-MAT (4.19M vertices, ~128M CSR entries, weights U(1,10), labels 0..4):
* Node2Vec p=0.5 q=2.0, one walker per vertex, L=80, in the launch configuration the
  benchmark times (default plan, autotuned rho), for AUTO, eRVS-only and eRJS-only;
* MetaPath schema (0,1,2,3,4) repeated, 1M uniform starts (seed 42), L=40.
The oracle replays a seeded sample of walkers (same walker ids, so the same random
streams) and every walk of the launch is checked to step along edges, to match the
schema, and to pad with -1.
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
    gg = GpuGraph(g22)
    yield gg
    gg.close()


@pytest.fixture(scope="module")
def og22(g22):
    og = oracle.Graph(g22)
    og.aux()
    return og


def _sample(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(k, n), replace=False)).astype(np.int64)


@pytest.mark.parametrize("strategy,k", [(oracle.AUTO, 65536), (oracle.RJS_ONLY, 65536), (oracle.RVS_ONLY, 1024)],
                         ids=["auto", "rjs", "rvs"])
def test_node2vec_scale22(g22, gg22, og22, strategy, k):
    tuned = fw.fw_plan_autotune(gg22.handle, fw.fw_logic_node2vec(0.5, 2.0, True))
    pl = oracle.Plan(rho=tuned.rho, d_lo=tuned.d_lo, rjs_cap=tuned.rjs_cap)
    starts = synth.all_vertices(g22["nv"])
    p, ln, st = gpu_walk(gg22, N2V, pl, strategy, starts, 80, 42)
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


def test_metapath_scale22(g22, gg22, og22):
    tuned = fw.fw_plan_autotune(gg22.handle, fw.fw_logic_metapath([0, 1, 2, 3, 4], True))
    pl = oracle.Plan(rho=tuned.rho, rjs_cap=tuned.rjs_cap)
    starts = synth.uniform_starts(g22["nv"], 1 << 20, 42)
    p, ln, st = gpu_walk(gg22, MP, pl, oracle.AUTO, starts, 40, 42)
    ok, pad_ok, (pos, taken) = edge_check_torch(g22, p, ln)
    assert ok and pad_ok
    # schema: the label of the edge taken at step j is schema[j mod 5]
    lab = torch.from_numpy(g22["label"]).to(pos.device)
    jj = torch.arange(40, device=pos.device)[None, :].expand(taken.shape[0], 40)[taken]
    assert bool((lab[pos] == (jj % 5).to(lab.dtype)).all().item())
    assert st["ended_early"] > 0
    sub = _sample(len(starts), 65536, 99)
    ora = oracle.walk(og22, MP, pl, oracle.AUTO, starts[sub], 40, 42, walker_ids=sub)
    rep = parity(p[sub], ln[sub], ora)
    print("metapath22", {k2: (v if not isinstance(v, list) else len(v)) for k2, v in rep.items()}, st)
    assert_parity(rep)
