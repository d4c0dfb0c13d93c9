"""The walk server: continuous batching against a resident graph (needs an MI355X).

Requests of mixed logic, size and length arrive from another thread while others run;
every result must be identical to the same request run alone with fw_walk and match the
oracle; the HBM budget must queue requests (never fail them) and the waiting queue must
push back with FW_E_BUSY when full.
"""
from __future__ import annotations

import threading
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import GpuGraph, assert_parity, fw_logic, gpu_walk, parity

import paper_2512_00705_amd as fw

pytestmark = pytest.mark.gpu
PLAN = oracle.Plan(rho=4.0, rjs_cap=64)


@pytest.fixture(scope="module")
def g12():
    return synth.rmat(12, 8 << 12, seed=1, nlabels=5)


@pytest.fixture(scope="module")
def gg12(g12):
    gg = GpuGraph(g12)
    yield gg
    gg.close()


def _requests(nv, k, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        if i % 3 == 2:
            lg = oracle.Logic(kind=oracle.METAPATH, weighted=bool(i % 2),
                              schema=tuple(int(x) for x in rng.integers(0, 5, 1 + i % 5)))
        elif i % 6 == 1:
            lg = oracle.Logic(kind=oracle.SECOND_PR, weighted=bool(i % 4 != 1), gamma=float(rng.choice([0.0, 0.2, 0.9])))
        else:
            lg = oracle.Logic(kind=oracle.NODE2VEC, weighted=bool(i % 4 != 1), p=float(rng.choice([0.25, 1, 4])),
                              q=float(rng.choice([0.5, 2])))
        n = int(np.floor(np.exp(rng.uniform(0, np.log(600)))))
        L = int(rng.integers(0, 40))
        starts = rng.integers(0, nv, n).astype(np.int32)
        out.append((lg, starts, L, 1000 + i))
    return out


def _serve_all(srv, reqs, gap_s=0.0):
    ids = {}

    def submit():
        for k, (lg, st, L, seed) in enumerate(reqs):
            ids[fw.fw_server_submit(srv, fw_logic(lg), st, L, seed)] = k
            if gap_s:
                time.sleep(gap_s)

    th = threading.Thread(target=submit)
    th.start()
    results = {}
    deadline = time.time() + 120
    while len(results) < len(reqs) and time.time() < deadline:
        rid = fw.fw_server_next_done(srv, 200)
        if rid:
            while rid not in ids:  # the submitter may not have recorded the id yet
                time.sleep(0.001)
            k = ids[rid]
            lg, st, L, seed = reqs[k]
            results[k] = fw.fw_server_result(srv, rid, len(st), L)
    th.join()
    return results


@pytest.mark.parametrize("tick_steps", [1, 7, 64])
def test_mix_equals_alone_and_oracle(g12, gg12, tick_steps):
    reqs = _requests(g12["nv"], 90, tick_steps)
    srv = fw.fw_server_create(gg12.handle, fw.fw_plan_default(rho=PLAN.rho, rjs_cap=PLAN.rjs_cap), fw.FW_AUTO,
                              64 << 20, tick_steps=tick_steps, max_active=64)
    try:
        results = _serve_all(srv, reqs, gap_s=0.0005)
        stats = fw.fw_server_stats(srv)
    finally:
        fw.fw_server_destroy(srv)
    assert len(results) == len(reqs)
    assert stats["finished"] == len(reqs) and stats["bytes_in_use"] == 0
    og = oracle.Graph(g12)
    for k, (lg, st, L, seed) in enumerate(reqs):
        p, ln, lat = results[k]
        alone = gpu_walk(gg12, lg, PLAN, oracle.AUTO, st, L, seed)
        np.testing.assert_array_equal(p, alone[0], err_msg=f"request {k}")
        np.testing.assert_array_equal(ln, alone[1], err_msg=f"request {k}")
        assert lat > 0
        if k % 6 == 0:
            assert_parity(parity(p, ln, oracle.walk(og, lg, PLAN, oracle.AUTO, st, L, seed)))


def test_budget_queues_and_busy(g12, gg12):
    # one long request holds most of a 2 MiB budget; later ones must wait, not fail
    rng = np.random.default_rng(3)
    big = (oracle.Logic(kind=oracle.NODE2VEC, p=1.0, q=1.0), rng.integers(0, g12["nv"], 400).astype(np.int32), 1000, 1)
    small = [(oracle.Logic(kind=oracle.NODE2VEC, p=2.0, q=0.5), rng.integers(0, g12["nv"], 300).astype(np.int32), 300,
              10 + i) for i in range(2)]
    srv = fw.fw_server_create(gg12.handle, fw.fw_plan_default(rho=4.0), fw.FW_AUTO, 2 << 20, tick_steps=1,
                              max_active=8, max_pending=2)
    try:
        with pytest.raises(fw.FlexiWalkError):  # can never fit the budget
            fw.fw_server_submit(srv, fw_logic(big[0]), np.zeros(5000, np.int32), 200, 0)
        ids = [fw.fw_server_submit(srv, fw_logic(big[0]), big[1], big[2], big[3])]
        for _ in range(2000):  # until the long request holds its block
            if fw.fw_server_stats(srv)["active"] >= 1:
                break
            time.sleep(0.001)
        ids += [fw.fw_server_submit(srv, fw_logic(lg), st, L, sd) for lg, st, L, sd in small]
        time.sleep(0.01)
        st = fw.fw_server_stats(srv)
        assert st["waiting"] >= 1  # held back by the budget while the long walk runs
        waiting_full = False
        try:
            for i in range(4):
                fw.fw_server_submit(srv, fw_logic(small[0][0]), small[0][1], 300, 99 + i)
        except fw.FlexiWalkError as e:
            waiting_full = e.code == fw.FW_E_BUSY
        assert waiting_full
        done = set()
        deadline = time.time() + 60
        while len(done) < 3 and time.time() < deadline:
            rid = fw.fw_server_next_done(srv, 200)
            if rid in ids:
                done.add(rid)
        assert done == set(ids)
        p, ln, _ = fw.fw_server_result(srv, ids[0], 400, 1000)
        alone = gpu_walk(gg12, big[0], oracle.Plan(rho=4.0), oracle.AUTO, big[1], 1000, 1)
        np.testing.assert_array_equal(p, alone[0])
    finally:
        fw.fw_server_destroy(srv)


def test_bad_start_and_teardown(g12, gg12):
    srv = fw.fw_server_create(gg12.handle, fw.fw_plan_default(), fw.FW_AUTO, 16 << 20, tick_steps=4)
    try:
        # a start outside [0, nv) is refused at submit; nothing is queued and the graph's
        # device error flag stays clear
        for bad in (g12["nv"] + 5, -1):
            with pytest.raises(fw.FlexiWalkError) as e:
                fw.fw_server_submit(srv, fw.fw_logic_node2vec(1.0, 1.0, True), np.array([3, bad, 9], np.int32), 6, 5)
            assert e.value.code == fw.FW_E_INVALID
        st = np.array([3, 7, 9], np.int32)
        rid = fw.fw_server_submit(srv, fw.fw_logic_node2vec(1.0, 1.0, True), st, 6, 5)
        got = 0
        for _ in range(100):
            got = fw.fw_server_next_done(srv, 100)
            if got:
                break
        assert got == rid
        p, ln, _ = fw.fw_server_result(srv, rid, 3, 6)
        alone = gpu_walk(gg12, oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=1.0, q=1.0), oracle.Plan(),
                         oracle.AUTO, st, 6, 5)
        np.testing.assert_array_equal(p, alone[0])
        fw.fw_graph_check(gg12.handle)
        with pytest.raises(fw.FlexiWalkError):  # results are handed out once
            fw.fw_server_result(srv, rid, 3, 6)
        for i in range(20):  # left running at teardown
            fw.fw_server_submit(srv, fw.fw_logic_node2vec(1.0, 1.0, True), np.arange(200, dtype=np.int32), 30, i)
    finally:
        fw.fw_server_destroy(srv)


@pytest.mark.parametrize("tick_steps", [1, 5])
@pytest.mark.parametrize("bound", [1, 2], ids=["split", "member"])
def test_split_bound_resume(g12, gg12, tick_steps, bound):
    """Walks suspended every few steps under the split bound (or the member board): a
    resumed walker recovers h(prev, cur) from the graph, so its samples equal an
    uninterrupted walk's."""
    pl = oracle.Plan(rho=1.0, rjs_cap=64, bound=bound)
    rng = np.random.default_rng(tick_steps)
    reqs = []
    for i in range(12):
        lg = oracle.Logic(kind=oracle.NODE2VEC, weighted=bool(i % 3), p=float(rng.choice([0.25, 0.5, 2.0])), q=2.0)
        reqs.append((lg, rng.integers(0, g12["nv"], int(rng.integers(1, 400))).astype(np.int32),
                     int(rng.integers(1, 30)), 500 + i))
    srv = fw.fw_server_create(gg12.handle, fw.fw_plan_default(rho=pl.rho, rjs_cap=pl.rjs_cap, bound=bound),
                              fw.FW_AUTO, 64 << 20, tick_steps=tick_steps, max_active=8)
    try:
        results = _serve_all(srv, reqs)
    finally:
        fw.fw_server_destroy(srv)
    og = oracle.Graph(g12)
    for k, (lg, st, L, seed) in enumerate(reqs):
        p, ln, _ = results[k]
        alone = gpu_walk(gg12, lg, pl, oracle.AUTO, st, L, seed)
        np.testing.assert_array_equal(p, alone[0], err_msg=f"request {k}")
        np.testing.assert_array_equal(ln, alone[1], err_msg=f"request {k}")
        assert_parity(parity(p, ln, oracle.walk(og, lg, pl, oracle.AUTO, st, L, seed)))


@pytest.mark.parametrize("bound", [1, 2], ids=["split", "member"])
def test_h_proposals_served(g12, bound):
    """Served walks under h-proportional proposals and the split bound (or the member
    board), suspended every 3 steps, equal the same walks run alone and the oracle's."""
    gg = GpuGraph(g12, index=True, alias=True)
    pl = oracle.Plan(rho=1.0, rjs_cap=64, bound=bound, proposal=1)
    rng = np.random.default_rng(9)
    reqs = [(oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=float(rng.choice([0.25, 2.0])), q=2.0),
             rng.integers(0, g12["nv"], int(rng.integers(1, 300))).astype(np.int32), int(rng.integers(1, 25)), 700 + i)
            for i in range(10)]
    srv = fw.fw_server_create(gg.handle,
                              fw.fw_plan_default(rho=pl.rho, rjs_cap=pl.rjs_cap, bound=bound, proposal=1),
                              fw.FW_AUTO, 64 << 20, tick_steps=3, max_active=8)
    try:
        results = _serve_all(srv, reqs)
    finally:
        fw.fw_server_destroy(srv)
    og = oracle.Graph(g12)
    try:
        for k, (lg, st, L, seed) in enumerate(reqs):
            p, ln, _ = results[k]
            alone = gpu_walk(gg, lg, pl, oracle.AUTO, st, L, seed)
            np.testing.assert_array_equal(p, alone[0], err_msg=f"request {k}")
            np.testing.assert_array_equal(ln, alone[1], err_msg=f"request {k}")
            assert_parity(parity(p, ln, oracle.walk(og, lg, pl, oracle.AUTO, st, L, seed)))
    finally:
        gg.close()


@pytest.mark.parametrize("tick_steps", [3, 64])
def test_label_proposals_served(g12, tick_steps):
    """The served configuration's plan kind: label-conditioned proposals for MetaPath and
    h-proportional ones for Node2Vec under the member board, requests suspended every few
    steps; each result equals the same request run alone and the oracle's walks."""
    gg = GpuGraph(g12, alias=True, label_alias=True)
    pl = oracle.Plan(rho=1.0, rjs_cap=64, bound=2, proposal=2)
    rng = np.random.default_rng(40 + tick_steps)
    reqs = []
    for i in range(16):
        if i % 2:
            lg = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2, 3, 4))
        else:
            lg = oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=float(rng.choice([0.25, 2.0])), q=2.0)
        reqs.append((lg, rng.integers(0, g12["nv"], int(rng.integers(1, 300))).astype(np.int32),
                     int(rng.integers(1, 40)), 900 + i))
    try:
        srv = fw.fw_server_create(gg.handle, fw.fw_plan_default(rho=pl.rho, rjs_cap=pl.rjs_cap, bound=2, proposal=2),
                                  fw.FW_AUTO, 64 << 20, tick_steps=tick_steps, max_active=8)
        try:
            results = _serve_all(srv, reqs)
        finally:
            fw.fw_server_destroy(srv)
        og = oracle.Graph(g12)
        for k, (lg, st, L, seed) in enumerate(reqs):
            p, ln, _ = results[k]
            alone = gpu_walk(gg, lg, pl, oracle.AUTO, st, L, seed)
            np.testing.assert_array_equal(p, alone[0], err_msg=f"request {k}")
            np.testing.assert_array_equal(ln, alone[1], err_msg=f"request {k}")
            assert_parity(parity(p, ln, oracle.walk(og, lg, pl, oracle.AUTO, st, L, seed)))
    finally:
        gg.close()
