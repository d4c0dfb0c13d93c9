"""Pins of the CPU oracle to the paper and to mathematics (no GPU).

Each test checks the oracle against something other than itself: values printed in
the paper (the worked example), published Philox answers, closed forms of Markov
chains, brute-force path enumeration, and the theorems the paper proves (eRJS bound
invariance, exponential-key and jump equivalence).  The last group plants known
mistakes in the oracle and shows that these pins catch them.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import exact
from tests._helpers import (assert_chisq, chisq_pvalue, hub_ring_graph, path_counts, triangle_graph,
                            worked_example_graph)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
P_BAD = 1e-8  # a planted mistake must fail far below it (a correct sampler passes at p > 0.01,
              # assert_chisq; fixed seeds: deterministic)

N2V = dict(kind=oracle.NODE2VEC, weighted=True, p=2.0, q=0.5)


def _walk_counts(g, logic, plan, strategy, start, L, n, seed=42):
    og = oracle.Graph(g)
    r = oracle.walk(og, logic, plan, strategy, np.full(n, start, np.int32), L, seed, diagnostics=False)
    return path_counts(r.paths), r


# ------------------------------------------------------------------ Philox, uniforms
def test_philox_published_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox(v[0:4], v[4:6])
        assert out.tolist() == v[6:10]


def test_uniform_exact_open_symmetric():
    lo, hi = oracle.uniform(0), oracle.uniform(0xFFFFFFFF)
    assert lo == 2.0 ** -24 and hi == 1.0 - 2.0 ** -24
    rng = np.random.default_rng(0)
    for x in rng.integers(0, 2 ** 32, 2000, dtype=np.uint64):
        u = oracle.uniform(int(x))
        m = int(x) >> 9
        assert Fraction(u) == Fraction(2 * m + 1, 2 ** 24)  # exact in float32
        assert 0.0 < u < 1.0
        # symmetric: complementing the top 23 bits mirrors u about 1/2
        assert oracle.uniform(int(x) ^ 0xFFFFFE00) == 1.0 - u


# ------------------------------------------------------------------ plain definition
def test_worked_example_exact():
    """Section 2.2 worked example: weights {3,2,4,1} -> {0.3,0.2,0.4,0.1}."""
    with open(os.path.join(GOLDEN, "worked_example.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    g = worked_example_graph()
    t = exact.transition(g, oracle.Logic(**N2V), 0, -1, 0)  # first step: static walk
    for nb, w, p in rows:
        assert t[int(nb)] == Fraction(p)


def test_node2vec_case_table():
    """Eq. node2vec: weights 1/a, 1, 1/b for dist 0, 1, 2 (hand-computed state)."""
    g = triangle_graph()
    # state prev=0, cur=1; N(1) = {0, 2, 3}; 0 is prev, 2 in N(0), 3 not in N(0)
    # h(1,0)=1, h(1,2)=3, h(1,3)=4 ; a=2, b=0.5 -> 1/2*1, 1*3, 2*4 = 0.5, 3, 8
    t = exact.transition(g, oracle.Logic(**N2V), 1, 0, 1)
    tot = Fraction(1, 2) + 3 + 8
    assert t == {0: Fraction(1, 2) / tot, 2: Fraction(3) / tot, 3: Fraction(8) / tot}
    # unweighted: 1/2, 1, 2
    t = exact.transition(g, oracle.Logic(kind=oracle.NODE2VEC, weighted=False, p=2.0, q=0.5), 1, 0, 1)
    assert t == {0: Fraction(1, 7), 2: Fraction(2, 7), 3: Fraction(4, 7)}


def test_metapath_schema_rule():
    g = triangle_graph(labels=True)
    lg = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2))
    # N(2) = {0 (lab 1, h 2), 1 (lab 2, h 3), 3 (lab 1, h 1), 4 (lab 0, h 3)}
    assert exact.transition(g, lg, 0, -1, 2) == {4: Fraction(1)}
    assert exact.transition(g, lg, 1, -1, 2) == {0: Fraction(2, 3), 3: Fraction(1, 3)}
    assert exact.transition(g, lg, 5, -1, 2) == {1: Fraction(1)}      # schema repeats: 5 % 3 = 2
    assert exact.transition(g, lg, 0, -1, 6) == {}                    # isolated vertex: walk ends


def test_enumeration_matches_matrix_power():
    """p = q = 1 makes Node2Vec first order: k-step marginals equal e_s P^k."""
    g = triangle_graph()
    lg = oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=1.0, q=1.0)
    P = exact.first_order_matrix(g)
    for start in (0, 3, 5):
        dist = exact.path_distribution(g, lg, start, 4)
        assert sum(dist.values()) == 1
        for k in range(1, 5):
            marg = np.zeros(g["nv"])
            for path, pr in dist.items():
                marg[path[k]] += float(pr)
            want = np.linalg.matrix_power(P, k)[start]
            np.testing.assert_allclose(marg, want, rtol=0, atol=1e-12)


def test_hmax_hsum_preprocess():
    g = synth.rmat(10, 8 << 10, seed=5)
    hmax, hsum = oracle.Graph(g).aux()
    rp, h = g["row_ptr"], g["h"].astype(np.float64)
    for v in range(g["nv"]):
        seg = h[rp[v]:rp[v + 1]]
        assert hmax[v] == (np.float32(seg.max()) if seg.size else 0.0)
        assert hsum[v] == np.float32(math.fsum(seg))  # double sum of these values is exact


# ------------------------------------------------------------------ samplers vs definition
STRATS = [
    ("auto", oracle.AUTO, oracle.Plan(rho=2.0, lanes=2)),
    ("rvs_P1", oracle.RVS_ONLY, oracle.Plan(lanes=1)),
    ("rvs_P2", oracle.RVS_ONLY, oracle.Plan(lanes=2)),
    ("rvs_P64", oracle.RVS_ONLY, oracle.Plan(lanes=64)),
    ("rvs_P2_share", oracle.RVS_ONLY, oracle.Plan(lanes=2, rvs_share=True)),
    ("rvs_nojump", oracle.RVS_ONLY, oracle.Plan(jump=False)),
    ("rjs", oracle.RJS_ONLY, oracle.Plan()),
    ("rjs_x4", oracle.RJS_ONLY, oracle.Plan(bound_scale=4.0)),
    ("rjs_x64", oracle.RJS_ONLY, oracle.Plan(bound_scale=64.0)),
    ("rjs_cap1", oracle.RJS_ONLY, oracle.Plan(rjs_cap=1, lanes=2)),
    ("its", oracle.ITS, oracle.Plan()),
]


@pytest.mark.parametrize("name,strategy,plan", STRATS, ids=[s[0] for s in STRATS])
def test_worked_example_sampled(name, strategy, plan):
    g = worked_example_graph()
    n = 40000
    probs = {(0, v): Fraction(p) for v, p in ((1, "0.3"), (2, "0.2"), (3, "0.4"), (4, "0.1"))}
    assert_chisq(lambda s: chisq_pvalue(_walk_counts(g, oracle.Logic(**N2V), plan, strategy, 0, 1, n, seed=s)[0],
                                        probs, n), 42, name)


@pytest.mark.parametrize("name,strategy,plan", STRATS, ids=[s[0] for s in STRATS])
def test_node2vec_paths_chisquare(name, strategy, plan):
    g = triangle_graph()
    lg = oracle.Logic(**N2V)
    n = 60000
    for start in (0, 4):
        probs = exact.path_distribution(g, lg, start, 3)
        assert_chisq(lambda s: chisq_pvalue(_walk_counts(g, lg, plan, strategy, start, 3, n, seed=s)[0], probs, n),
                     7 + start, (name, start))


@pytest.mark.parametrize("strategy", [oracle.AUTO, oracle.RVS_ONLY, oracle.RJS_ONLY])
def test_metapath_paths_chisquare(strategy):
    g = triangle_graph(labels=True)
    lg = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2))
    n = 40000
    plan = oracle.Plan(rho=1.0, lanes=2, rjs_cap=8)
    for start in (0, 2, 6):
        probs = exact.path_distribution(g, lg, start, 4)
        assert_chisq(lambda s: chisq_pvalue(_walk_counts(g, lg, plan, strategy, start, 4, n, seed=s)[0], probs, n),
                     11, start)


def _hub_case(plan, strategy, n=40000, seed=5):
    """Second step at the hub: prev = leaf 1, so N(hub) holds all three Node2Vec cases."""
    g = hub_ring_graph()
    lg = oracle.Logic(**N2V)
    og = oracle.Graph(g)
    r = oracle.walk(og, lg, plan, strategy, np.full(n, 1, np.int32), 2, seed, diagnostics=False)
    went_hub = r.paths[:, 1] == 0
    nxt = r.paths[went_hub, 2]
    counts = {}
    for v, c in zip(*np.unique(nxt, return_counts=True)):
        counts[int(v)] = int(c)
    probs = exact.transition(g, lg, 1, 1, 0)
    return chisq_pvalue(counts, probs, int(went_hub.sum())), r


@pytest.mark.parametrize("name,strategy,plan", [
    ("rvs_jump_P64", oracle.RVS_ONLY, oracle.Plan(lanes=64)),
    ("rvs_jump_P7", oracle.RVS_ONLY, oracle.Plan(lanes=7)),
    ("rvs_jump_P256", oracle.RVS_ONLY, oracle.Plan(lanes=256)),
    ("rvs_jump_P1024", oracle.RVS_ONLY, oracle.Plan(lanes=1024)),
    ("rvs_hub_bucket_P256", oracle.RVS_ONLY, oracle.Plan(hub_deg=600, hub_lanes=256)),
    ("rvs_share_P7", oracle.RVS_ONLY, oracle.Plan(lanes=7, rvs_share=True)),
    ("rvs_share_P64", oracle.RVS_ONLY, oracle.Plan(lanes=64, rvs_share=True)),
    ("rvs_share_P256", oracle.RVS_ONLY, oracle.Plan(lanes=256, rvs_share=True)),
    ("rvs_share_hub_bucket_P128", oracle.RVS_ONLY, oracle.Plan(hub_deg=600, hub_lanes=128, rvs_share=True)),
    ("rvs_nojump", oracle.RVS_ONLY, oracle.Plan(jump=False)),
    ("rjs", oracle.RJS_ONLY, oracle.Plan()),
])
def test_hub_distribution(name, strategy, plan):
    _, r = _hub_case(plan, strategy)
    assert_chisq(lambda s: _hub_case(plan, strategy, seed=s)[0], 5, name)
    if strategy == oracle.RVS_ONLY and plan.jump:
        # the jump skips most keys: far fewer key draws than items scanned
        assert r.counters["rvs_triggers"] < 0.2 * 600 * r.counters["steps"] / 2


def test_hub_lane_bucket_dispatch():
    """The degree bucket picks P per step: with hub_deg = 600 the hub's eRVS steps run with
    hub_lanes lanes and every other row with 64, so the walks equal those of a plan with
    P = 256 everywhere (rows of at most 64 entries are keyed in round 0 alone, which does not
    depend on P); one more than the hub's degree leaves every step at P = 64.  P itself
    changes the stream: the P = 256 and P = 64 walks differ."""
    g = hub_ring_graph()
    og = oracle.Graph(g)
    lg = oracle.Logic(**N2V)
    starts = np.arange(1, 601, dtype=np.int32)
    walk = lambda pl: oracle.walk(og, lg, pl, oracle.RVS_ONLY, starts, 6, 17, diagnostics=False).paths
    p64, p256 = walk(oracle.Plan(lanes=64)), walk(oracle.Plan(lanes=256))
    assert not np.array_equal(p64, p256)
    assert np.array_equal(walk(oracle.Plan(hub_deg=600, hub_lanes=256)), p256)
    assert np.array_equal(walk(oracle.Plan(hub_deg=601, hub_lanes=256)), p64)
    assert np.array_equal(walk(oracle.Plan(hub_deg=0, hub_lanes=256)), p64)


def test_rvs_share_draws_fewer_keys():
    """Sharing the largest threshold after each round with a jump event leaves fewer lanes
    able to pass it: at the 600-neighbour hub with 64 lanes the key draws per step fall by
    more than half (the sampler stays exact: test_hub_distribution)."""
    _, paper = _hub_case(oracle.Plan(lanes=64), oracle.RVS_ONLY)
    _, share = _hub_case(oracle.Plan(lanes=64, rvs_share=True), oracle.RVS_ONLY)
    assert share.counters["steps"] == paper.counters["steps"]
    assert share.counters["rvs_triggers"] < 0.5 * paper.counters["rvs_triggers"]


def test_rvs_share_cases_that_equal_the_paper_form():
    """Where no lane can hold a threshold below another's the shared form is the paper's
    bit for bit: one lane (P = 1), and rows of at most P entries (round 0 decides them)."""
    og = oracle.Graph(hub_ring_graph())
    lg = oracle.Logic(**N2V)
    starts = np.arange(0, 601, dtype=np.int32)
    walk = lambda pl: oracle.walk(og, lg, pl, oracle.RVS_ONLY, starts, 5, 23, diagnostics=False)
    a, b = walk(oracle.Plan(lanes=1)), walk(oracle.Plan(lanes=1, rvs_share=True))
    np.testing.assert_array_equal(a.paths, b.paths)
    assert a.counters == b.counters
    a, b = walk(oracle.Plan(lanes=1024)), walk(oracle.Plan(lanes=1024, rvs_share=True))
    np.testing.assert_array_equal(a.paths, b.paths)
    # with P = 64 the hub's scan differs
    a, b = walk(oracle.Plan(lanes=64)), walk(oracle.Plan(lanes=64, rvs_share=True))
    assert a.counters["rvs_triggers"] != b.counters["rvs_triggers"]


def _pin_rvs_share():
    for lanes in (7, 64):
        test_hub_distribution(f"share{lanes}", oracle.RVS_ONLY, oracle.Plan(lanes=lanes, rvs_share=True))


def test_rjs_mean_trials_and_known_bound():
    """Pr[accept] = 1/c (Section 3.3): mean trials = deg * B / sum w~.

    Unweighted Node2Vec with a = 1, b = 0.5 has max weight exactly 2 (Section 3.3),
    so B = 2 and the mean trial count pins the bound.
    """
    g = triangle_graph()
    for lg, B in ((oracle.Logic(kind=oracle.NODE2VEC, weighted=False, p=1.0, q=0.5), 2.0),
                  (oracle.Logic(**N2V), None)):
        og = oracle.Graph(g)
        hmax, _ = og.aux()
        n = 40000
        # state: prev = 0, cur = 1 (teacher-forced single step), walker ids distinct
        trials = np.empty(n)
        for i in range(n):
            nxt, m, kind, t = oracle.step_once(og, lg, oracle.Plan(rjs_cap=100000), oracle.RJS_ONLY, 3, i, 1, 0, 1)
            trials[i] = t
        t = exact.transition(g, lg, 1, 0, 1)
        ws = [exact.transition_weight(g, lg, 1, 0, k) for k in range(int(g["row_ptr"][1]), int(g["row_ptr"][2]))]
        bound = B if B is not None else 2.0 * float(hmax[1])
        want = len(ws) * bound / float(sum(ws))
        se = math.sqrt(want * (want - 1) / n)  # geometric distribution
        assert abs(trials.mean() - want) < 5 * se, (trials.mean(), want)


# ------------------------------------------------------------------ split bound (plan.bound = 1)
# p = 0.25 makes the return edge the heaviest (1/p = 4 > 1 > 1/q), so the extra column
# of the split bound is non-empty in most states
N2V_RET = dict(kind=oracle.NODE2VEC, weighted=True, p=0.25, q=2.0)
SPLIT = [
    ("rjs", oracle.RJS_ONLY, oracle.Plan(bound=1)),
    ("rjs_x4", oracle.RJS_ONLY, oracle.Plan(bound=1, bound_scale=4.0)),
    ("auto", oracle.AUTO, oracle.Plan(bound=1, rho=1.0, lanes=2)),
    ("rjs_cap1", oracle.RJS_ONLY, oracle.Plan(bound=1, rjs_cap=1, lanes=2)),
]


@pytest.mark.parametrize("name,strategy,plan", SPLIT, ids=[s[0] for s in SPLIT])
@pytest.mark.parametrize("logic", [N2V_RET, N2V, dict(N2V_RET, weighted=False)], ids=["ret", "n2v", "unweighted"])
def test_split_bound_paths_chisquare(name, strategy, plan, logic):
    """Any bound that dominates every w~ leaves the distribution of Eq. (prob) unchanged
    (Section 3.3): the split bound's walks follow the exact path distribution."""
    g = triangle_graph()
    lg = oracle.Logic(**logic)
    n = 60000
    for start in (0, 4):
        probs = exact.path_distribution(g, lg, start, 3)
        assert_chisq(lambda s: chisq_pvalue(_walk_counts(g, lg, plan, strategy, start, 3, n, seed=s)[0], probs, n),
                     11 + start, (name, start))


def test_split_bound_hub_distribution():
    """Second step at the 600-neighbour hub, where the return edge is one column of 600."""
    g = hub_ring_graph()
    lg = oracle.Logic(**N2V_RET)
    og = oracle.Graph(g)
    n = 40000

    def pval(seed):
        r = oracle.walk(og, lg, oracle.Plan(bound=1), oracle.RJS_ONLY, np.full(n, 1, np.int32), 2, seed,
                        diagnostics=False)
        went_hub = r.paths[:, 1] == 0
        counts = {int(v): int(c) for v, c in zip(*np.unique(r.paths[went_hub, 2], return_counts=True))}
        return chisq_pvalue(counts, exact.transition(g, lg, 1, 1, 0), int(went_hub.sum()))
    assert_chisq(pval, 5)


def test_split_bound_mean_trials():
    """Mean trials of the split board = (deg * Bn + E) / sum w~, against deg * B / sum w~
    for the paper's bound.  State prev = 3, cur = 1 of the triangle graph: N(1) = {0, 2, 3}
    with h = 1, 3, 4, so w~ = 0.5, 3, 16 (two hops, common neighbour, return), h_MAX = 4,
    Bn = max(1, 1/q) * 4 = 4, E = 16 - 4 = 12: 24 / 19.5 trials against 3 * 16 / 19.5."""
    g = triangle_graph()
    lg = oracle.Logic(**N2V_RET)
    og = oracle.Graph(g)
    og.aux()
    ws = [exact.transition_weight(g, lg, 1, 3, k) for k in range(int(g["row_ptr"][1]), int(g["row_ptr"][2]))]
    assert sorted(float(w) for w in ws) == [0.5, 3.0, 16.0]
    n = 40000
    for plan, want in ((oracle.Plan(bound=1, rjs_cap=100000), 24.0 / 19.5),
                       (oracle.Plan(bound=0, rjs_cap=100000), 48.0 / 19.5)):
        trials = np.empty(n)
        for i in range(n):
            trials[i] = oracle.step_once(og, lg, plan, oracle.RJS_ONLY, 3, i, 1, 3, 1)[3]
        se = math.sqrt(want * (want - 1) / n)
        assert abs(trials.mean() - want) < 5 * se, (plan.bound, trials.mean(), want)


def test_split_bound_is_paper_bound_without_excess():
    """With 1/p <= max(1, 1/q) the extra column is empty and Bn is the paper's bound,
    so eRJS-only walks draw exactly the same samples under both settings."""
    g = synth.rmat(10, 8 << 10, seed=4)
    og = oracle.Graph(g)
    lg = oracle.Logic(**N2V)
    st = np.arange(g["nv"], dtype=np.int32)
    a = oracle.walk(og, lg, oracle.Plan(bound=0), oracle.RJS_ONLY, st, 12, 9, diagnostics=False)
    b = oracle.walk(og, lg, oracle.Plan(bound=1), oracle.RJS_ONLY, st, 12, 9, diagnostics=False)
    np.testing.assert_array_equal(a.paths, b.paths)
    assert a.counters["rjs_trials"] == b.counters["rjs_trials"]


def test_split_bound_fewer_trials_rmat():
    """On a skewed graph the split board needs fewer trials per step than the paper's
    bound when the return weight dominates (the reason it exists)."""
    g = synth.rmat(12, 8 << 12, seed=2)
    og = oracle.Graph(g)
    lg = oracle.Logic(**N2V_RET)
    st = np.arange(g["nv"], dtype=np.int32)
    a = oracle.walk(og, lg, oracle.Plan(bound=0), oracle.RJS_ONLY, st, 20, 9, diagnostics=False)
    b = oracle.walk(og, lg, oracle.Plan(bound=1), oracle.RJS_ONLY, st, 20, 9, diagnostics=False)
    ta = a.counters["rjs_trials"] / a.counters["steps"]
    tb = b.counters["rjs_trials"] / b.counters["steps"]
    assert tb < 0.75 * ta, (ta, tb)


# ------------------------------------------------------------------ second-order PageRank
PR2 = dict(kind=oracle.SECOND_PR, weighted=True, gamma=0.25)


def test_second_pr_hand_worked_state():
    """Eq. (2ndpr) at prev = 2 (degree 4), cur = 1 (degree 3) of the triangle graph with
    gamma = 1/4: max_d = 4, weight (3/4 / 3 + 1/4 / 4) * 4 = 5/4 for u in N(2) and
    (3/4 / 3) * 4 = 1 otherwise (the return edge to 2 included).  N(1) = {0, 2, 3} with
    h = 1, 3, 4 gives w~ = 5/4, 3, 5 and probabilities 5/37, 12/37, 20/37."""
    g = triangle_graph()
    lg = oracle.Logic(**PR2)
    t = exact.transition(g, lg, 1, 2, 1)
    assert t == {0: Fraction(5, 37), 2: Fraction(12, 37), 3: Fraction(20, 37)}
    assert exact.transition(g, lg, 0, -1, 1) == {0: Fraction(1, 8), 2: Fraction(3, 8), 3: Fraction(4, 8)}


@pytest.mark.parametrize("name,strategy,plan", STRATS, ids=[s[0] for s in STRATS])
@pytest.mark.parametrize("gamma", [0.25, 0.7])
def test_second_pr_paths_chisquare(name, strategy, plan, gamma):
    g = triangle_graph()
    lg = oracle.Logic(**dict(PR2, gamma=gamma))
    n = 60000
    for start in (0, 4):
        probs = exact.path_distribution(g, lg, start, 3)
        assert_chisq(lambda s: chisq_pvalue(_walk_counts(g, lg, plan, strategy, start, 3, n, seed=s)[0], probs, n),
                     31 + start, (name, start))


def test_second_pr_gamma0_is_first_order():
    """gamma = 0 makes both branches (1/d(v)) * max_d: the step is the static walk
    p(u) = h(v, u) / sum h, i.e. a row of the first-order transition matrix."""
    g = hub_ring_graph(40)
    lg = oracle.Logic(**dict(PR2, gamma=0.0))
    og = oracle.Graph(g)
    P = exact.first_order_matrix(g)
    n = 80000
    probs = {u: Fraction(float(P[0, u])) for u in range(g["nv"]) if P[0, u] > 0}
    for strategy in (oracle.RJS_ONLY, oracle.RVS_ONLY):
        def pval(seed):
            r = oracle.walk(og, lg, oracle.Plan(), strategy, np.full(n, 3, np.int32), 2, seed, diagnostics=False)
            at_hub = r.paths[:, 1] == 0
            counts = {int(v): int(c) for v, c in zip(*np.unique(r.paths[at_hub, 2], return_counts=True))}
            return chisq_pvalue(counts, probs, int(at_hub.sum()))
        assert_chisq(pval, 17, strategy)


def test_second_pr_mean_trials():
    """State prev = 2, cur = 1 (gamma = 1/4): B = max(w) * h_MAX = 5/4 * 4 = 5, so the mean
    eRJS trial count is deg * B / sum w~ = 3 * 5 / (37/4) = 60/37."""
    g = triangle_graph()
    lg = oracle.Logic(**PR2)
    og = oracle.Graph(g)
    og.aux()
    n = 40000
    trials = np.array([oracle.step_once(og, lg, oracle.Plan(rjs_cap=100000), oracle.RJS_ONLY, 3, i, 1, 2, 1)[3]
                       for i in range(n)], dtype=np.float64)
    want = 60.0 / 37.0
    se = math.sqrt(want * (want - 1) / n)
    assert abs(trials.mean() - want) < 5 * se, (trials.mean(), want)


# ------------------------------------------------------------------ h-proportional proposals
def _alias_distribution(g, thr, idx, v):
    """Exact probabilities with which a uniform slot plus the alias coin yields each
    offset of row v: slot s keeps itself with thr_s / 2^32, else yields idx_s."""
    b, n = int(g["row_ptr"][v]), int(g["row_ptr"][v + 1] - g["row_ptr"][v])
    P = [Fraction(0)] * n
    for s in range(n):
        keep = Fraction(int(thr[b + s]), 1 << 32)
        P[s] += keep / n
        P[int(idx[b + s])] += (1 - keep) / n
    return P


@pytest.mark.parametrize("weights", ["triangle", "hub", "pareto1", "pareto3"])
def test_alias_tables_realise_h(weights):
    """Each row's alias table draws offset k with probability h_k / sum h, to within the
    2^-32 granularity of the thresholds (Walker's alias method)."""
    if weights == "triangle":
        g = triangle_graph()
    elif weights == "hub":
        g = hub_ring_graph(600)
    else:
        g = synth.rmat(9, 8 << 9, seed=3)
        g["h"] = synth.pareto_weights(g["row_ptr"], g["col"], float(weights[6:]), 5)
    og = oracle.Graph(g)
    thr, idx = og.alias()
    rows = range(g["nv"]) if g["nv"] <= 700 else np.random.default_rng(0).choice(g["nv"], 120, replace=False)
    for v in rows:
        b, e = int(g["row_ptr"][v]), int(g["row_ptr"][v + 1])
        if e == b:
            continue
        h = [Fraction(float(x)) for x in g["h"][b:e]]
        H = sum(h)
        got = _alias_distribution(g, thr, idx, int(v))
        assert sum(got) == 1
        for k in range(e - b):
            assert abs(got[k] - h[k] / H) <= Fraction(e - b + 2, 1 << 31), (v, k)


def _labelled_rmat(scale, seed, weights="uniform"):
    g = synth.rmat(scale, 8 << scale, seed=seed, nlabels=5)
    if weights != "uniform":
        g["h"] = synth.pareto_weights(g["row_ptr"], g["col"], float(weights[6:]), seed)
    return g


@pytest.mark.parametrize("weights", ["triangle", "uniform", "pareto1"])
def test_label_groups_realise_h(weights):
    """Label-conditioned proposals: group (v, l) holds exactly the entries of row v with
    label l, in row order, starting where the groups of the smaller labels end; its alias
    table draws each of them with probability h / (sum of h over the group), to within the
    2^-32 granularity of the thresholds."""
    g = triangle_graph(labels=True) if weights == "triangle" else _labelled_rmat(9, 3, weights)
    og = oracle.Graph(g)
    nlab, lrow, lperm, lthr, lalias = og.label_alias()
    assert nlab == int(g["label"].max()) + 1 and lrow[g["nv"] * nlab] == g["ne"]
    rows = range(g["nv"]) if g["nv"] <= 700 else np.random.default_rng(1).choice(g["nv"], 150, replace=False)
    for v in rows:
        b, e = int(g["row_ptr"][v]), int(g["row_ptr"][v + 1])
        assert lrow[v * nlab] == b and lrow[(v + 1) * nlab] == e if v + 1 < g["nv"] else lrow[v * nlab] == b
        for lab in range(nlab):
            g0, g1 = int(lrow[v * nlab + lab]), int(lrow[v * nlab + lab + 1])
            want = [k for k in range(e - b) if g["label"][b + k] == lab]
            assert list(lperm[g0:g1]) == want, (v, lab)
            if g1 == g0:
                continue
            n = g1 - g0
            P = [Fraction(0)] * n
            for t in range(n):
                keep = Fraction(int(lthr[g0 + t]), 1 << 32)
                P[t] += keep / n
                P[int(lalias[g0 + t])] += (1 - keep) / n
            assert sum(P) == 1
            h = [Fraction(float(g["h"][b + k])) for k in want]
            H = sum(h)
            for t in range(n):
                assert abs(P[t] - h[t] / H) <= Fraction(n + 2, 1 << 31), (v, lab, t)


MP_L = dict(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2))
MP_LAB = [("rjs", oracle.RJS_ONLY, oracle.Plan(proposal=2)),
          ("auto", oracle.AUTO, oracle.Plan(proposal=2, rho=2.5, lanes=2)),
          ("auto_dlo", oracle.AUTO, oracle.Plan(proposal=2, rho=0.5, d_lo=3, lanes=2)),
          ("random", oracle.RANDOM_SELECT, oracle.Plan(proposal=2, lanes=2))]


@pytest.mark.parametrize("name,strategy,plan", MP_LAB, ids=[s[0] for s in MP_LAB])
def test_label_proposals_paths_chisquare(name, strategy, plan):
    """MetaPath paths with label-conditioned proposals against the exact path
    probabilities (triangle graph with labels, two starts, three steps)."""
    g = triangle_graph(labels=True)
    lg = oracle.Logic(**MP_L)
    n = 60000
    for start in (0, 4):
        probs = exact.path_distribution(g, lg, start, 3)
        assert_chisq(lambda s: chisq_pvalue(_walk_counts(g, lg, plan, strategy, start, 3, n, seed=s)[0], probs, n),
                     13 + start, (name, start))


def test_label_proposals_one_trial_and_valid_walks():
    """Every eRJS step of a label-conditioned plan takes one trial; every step follows an
    edge with the schema's label; a walk ends exactly where the current vertex has no
    neighbour with the wanted label (all weights here are positive)."""
    g = _labelled_rmat(10, 7)
    og = oracle.Graph(g)
    lg = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2, 3, 4))
    starts = synth.uniform_starts(g["nv"], 3000, 5)
    r = oracle.walk(og, lg, oracle.Plan(proposal=2, rho=4.0), oracle.AUTO, starts, 12, 9)
    c = r.counters
    assert c["rjs_steps"] > 0 and c["rvs_steps"] > 0  # rows below rho go to eRVS
    assert c["rjs_trials"] == c["rjs_steps"] and c["rjs_fallbacks"] == 0
    rp, col, lab = g["row_ptr"], g["col"], g["label"]
    for p, n in zip(r.paths, r.lengths):
        for j in range(n):
            row = range(int(rp[p[j]]), int(rp[p[j] + 1]))
            assert any(col[k] == p[j + 1] and lab[k] == j % 5 for k in row)
        if n < 12:
            assert not any(lab[k] == n % 5 for k in range(int(rp[p[n]]), int(rp[p[n] + 1])))


def test_label_proposals_zero_weight_group_ends_walk():
    """A group whose weights are all 0 holds no neighbour of positive weight: the walk ends
    there, under the label-conditioned proposal as under eRVS and uniform eRJS."""
    # vertex 0: label-0 neighbours 1, 2 with h = 0, a label-1 neighbour 3 with h = 5
    g = synth.csr_from_edges(4, [(0, 1), (0, 2), (0, 3)], h=[0.0, 0.0, 5.0], label=[0, 0, 1])
    og = oracle.Graph(g)
    lg = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1))
    st = np.zeros(50, np.int32)
    for strategy, plan in ((oracle.RJS_ONLY, oracle.Plan(proposal=2)), (oracle.RVS_ONLY, oracle.Plan(proposal=2)),
                           (oracle.RJS_ONLY, oracle.Plan())):
        r = oracle.walk(og, lg, plan, strategy, st, 3, 4)
        assert (r.lengths == 0).all(), (strategy, plan.proposal)
    lg1 = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(1, 0))
    r = oracle.walk(og, lg1, oracle.Plan(proposal=2), oracle.RJS_ONLY, st, 3, 4)
    # the label-1 step goes to 3; 3's only edge (back to 0) has label 1, so the label-0 step ends
    assert (r.paths[:, 1] == 3).all() and (r.lengths == 1).all()


N2V_H = [("rjs", oracle.RJS_ONLY, oracle.Plan(proposal=1)),
         ("rjs_split", oracle.RJS_ONLY, oracle.Plan(proposal=1, bound=1)),
         ("auto_split", oracle.AUTO, oracle.Plan(proposal=1, bound=1, rho=1.0, lanes=2)),
         ("rjs_cap1", oracle.RJS_ONLY, oracle.Plan(proposal=1, rjs_cap=1, lanes=2))]


@pytest.mark.parametrize("name,strategy,plan", N2V_H, ids=[s[0] for s in N2V_H])
@pytest.mark.parametrize("logic", [N2V, N2V_RET, PR2, dict(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2))],
                         ids=["n2v", "n2v_ret", "2ndpr", "metapath"])
def test_h_proposals_paths_chisquare(name, strategy, plan, logic):
    g = triangle_graph(labels=True)
    lg = oracle.Logic(**logic)
    n = 60000
    for start in (0, 4):
        probs = exact.path_distribution(g, lg, start, 3)
        assert_chisq(lambda s: chisq_pvalue(_walk_counts(g, lg, plan, strategy, start, 3, n, seed=s)[0], probs, n),
                     61 + start, (name, start))


def test_h_proposals_hub_and_skew():
    """The 600-neighbour hub, and Pareto(1) weights where uniform proposals need hundreds
    of trials per step: same exact distribution, far fewer trials."""
    g = hub_ring_graph(600)
    lg = oracle.Logic(**N2V_RET)
    og = oracle.Graph(g)
    n = 40000

    def pval(seed):
        r = oracle.walk(og, lg, oracle.Plan(proposal=1, bound=1), oracle.RJS_ONLY, np.full(n, 1, np.int32), 2, seed,
                        diagnostics=False)
        at_hub = r.paths[:, 1] == 0
        counts = {int(v): int(c) for v, c in zip(*np.unique(r.paths[at_hub, 2], return_counts=True))}
        return chisq_pvalue(counts, exact.transition(g, lg, 1, 1, 0), int(at_hub.sum()))
    assert_chisq(pval, 5)
    g = synth.rmat(12, 8 << 12, seed=2)
    g["h"] = synth.pareto_weights(g["row_ptr"], g["col"], 1.0, 3)
    og = oracle.Graph(g)
    st = np.arange(g["nv"], dtype=np.int32)
    u = oracle.walk(og, oracle.Logic(**N2V), oracle.Plan(rjs_cap=1 << 20), oracle.RJS_ONLY, st, 10, 9, diagnostics=False)
    a = oracle.walk(og, oracle.Logic(**N2V), oracle.Plan(proposal=1, rjs_cap=1 << 20), oracle.RJS_ONLY, st, 10, 9,
                    diagnostics=False)
    tu, ta = (x.counters["rjs_trials"] / x.counters["steps"] for x in (u, a))
    assert ta < 0.05 * tu and ta < 4.0, (tu, ta)


def test_h_proposals_mean_trials():
    """State prev = 3, cur = 1 of the triangle graph, p = 1/4, q = 2: w = 1/2, 1, 4 for
    u = 0, 2, 3 with h = 1, 3, 4 (sum 8), so sum w~ = 19.5.  With the split bound W = 1 and
    the return edge's extra column (4 - 1) * 4 = 12: trials = (1 * 8 + 12) / 19.5; with the
    paper's bound W = 4: trials = 4 * 8 / 19.5."""
    g = triangle_graph()
    lg = oracle.Logic(**N2V_RET)
    og = oracle.Graph(g)
    n = 40000
    for plan, want in ((oracle.Plan(proposal=1, bound=1, rjs_cap=100000), 20.0 / 19.5),
                       (oracle.Plan(proposal=1, bound=0, rjs_cap=100000), 32.0 / 19.5)):
        trials = np.array([oracle.step_once(og, lg, plan, oracle.RJS_ONLY, 3, i, 1, 3, 1)[3] for i in range(n)],
                          dtype=np.float64)
        se = math.sqrt(max(want * (want - 1), 1e-12) / n)
        assert abs(trials.mean() - want) < 5 * se + 1e-9, (plan.bound, trials.mean(), want)


# ------------------------------------------------------------------ member board (plan.bound = 2)
MB = [("rjs", oracle.RJS_ONLY, oracle.Plan(bound=2)),
      ("rjs_h", oracle.RJS_ONLY, oracle.Plan(bound=2, proposal=1)),
      ("auto_h", oracle.AUTO, oracle.Plan(bound=2, proposal=1, rho=1.0, lanes=2)),
      ("rjs_cap1", oracle.RJS_ONLY, oracle.Plan(bound=2, rjs_cap=1, lanes=2))]


@pytest.mark.parametrize("name,strategy,plan", MB, ids=[s[0] for s in MB])
@pytest.mark.parametrize("logic", [dict(kind=oracle.NODE2VEC, weighted=True, p=0.25, q=2.0),
                                   dict(kind=oracle.NODE2VEC, weighted=True, p=4.0, q=2.0),
                                   dict(kind=oracle.NODE2VEC, weighted=False, p=1.0, q=4.0), PR2,
                                   dict(PR2, gamma=0.7), dict(kind=oracle.NODE2VEC, weighted=True, p=2.0, q=0.5)],
                         ids=["n2v_ret", "n2v_p4", "n2v_unweighted", "2ndpr", "2ndpr_g07", "n2v_q05"])
def test_member_board_paths_chisquare(name, strategy, plan, logic):
    """The member board keeps the exact distribution: every proposal in the regular
    columns is taken at the lower weight, members get their excess from the member region
    and the return edge from its column (q <= 1 falls back to the split board)."""
    g = triangle_graph()
    lg = oracle.Logic(**logic)
    n = 60000
    for start in (0, 4):
        probs = exact.path_distribution(g, lg, start, 3)
        assert_chisq(lambda s: chisq_pvalue(_walk_counts(g, lg, plan, strategy, start, 3, n, seed=s)[0], probs, n),
                     71 + start, (name, start))


def test_member_board_hub():
    g = hub_ring_graph(600)
    og = oracle.Graph(g)
    n = 40000
    for logic in (N2V_RET, PR2):
        lg = oracle.Logic(**logic)
        for prop in (0, 1):
            def pval(seed):
                r = oracle.walk(og, lg, oracle.Plan(bound=2, proposal=prop), oracle.RJS_ONLY, np.full(n, 1, np.int32),
                                2, seed, diagnostics=False)
                at_hub = r.paths[:, 1] == 0
                counts = {int(v): int(c) for v, c in zip(*np.unique(r.paths[at_hub, 2], return_counts=True))}
                return chisq_pvalue(counts, exact.transition(g, lg, 1, 1, 0), int(at_hub.sum()))
            assert_chisq(pval, 5, (logic, prop))


def test_member_board_mean_trials():
    """Fan graph: v = 0 joined to 1..6 with h(0, u) = u, v' = 1 joined to 0 and 2.
    Second-order PageRank with gamma = 1/4 at d(v) = 6, d(v') = 2: w_in = 3/2, w_out = 3/4,
    one member (vertex 2), sum w~ = (3/4) * 21 + (3/4) * 2 = 69/4, h_MAX = 6.
    h-proportional: regular area (3/4) * 21 plus member region (3/4) * 6 * 2 = 99/4, so
    33/23 trials per step (the single-bound board, (3/2) * 21, would take 42/23);
    uniform: 6 * (3/4) * 6 + 9 = 36, 48/23 trials (single bound 54, 72/23)."""
    g = synth.csr_from_edges(7, [(0, 1), (0, 2), (0, 3), (0, 4), (0, 5), (0, 6), (1, 2)],
                             h=[1, 2, 3, 4, 5, 6, 1])
    lg = oracle.Logic(**PR2)
    og = oracle.Graph(g)
    n = 40000
    for bound, prop, want in ((2, 1, 33.0 / 23.0), (2, 0, 48.0 / 23.0), (0, 1, 42.0 / 23.0), (0, 0, 72.0 / 23.0)):
        plan = oracle.Plan(bound=bound, proposal=prop, rjs_cap=100000)
        trials = np.array([oracle.step_once(og, lg, plan, oracle.RJS_ONLY, 3, i, 1, 1, 0)[3] for i in range(n)],
                          dtype=np.float64)
        se = math.sqrt(want * (want - 1) / n)
        assert abs(trials.mean() - want) < 5 * se, (bound, prop, trials.mean(), want)


def test_member_board_fewer_trials_second_pr():
    """On a skewed graph second-order PageRank's bound (the larger branch) is loose when
    d(v) >> d(v'); the member board's area does not grow with d(v) / d(v')."""
    g = synth.rmat(12, 8 << 12, seed=2)
    og = oracle.Graph(g)
    lg = oracle.Logic(**PR2)
    st = np.arange(g["nv"], dtype=np.int32)
    a = oracle.walk(og, lg, oracle.Plan(proposal=1, rjs_cap=1 << 20), oracle.RJS_ONLY, st, 20, 9, diagnostics=False)
    b = oracle.walk(og, lg, oracle.Plan(proposal=1, bound=2, rjs_cap=1 << 20), oracle.RJS_ONLY, st, 20, 9,
                    diagnostics=False)
    ta, tb = (x.counters["rjs_trials"] / x.counters["steps"] for x in (a, b))
    assert tb < 0.4 * ta and tb < 2.0, (ta, tb)


# ------------------------------------------------------------------ comparison selection policies
@pytest.mark.parametrize("strategy", [oracle.RANDOM_SELECT, oracle.DEGREE_SELECT], ids=["random", "degree"])
@pytest.mark.parametrize("logic", [N2V, PR2], ids=["node2vec", "2ndpr"])
def test_selection_policies_exact(strategy, logic):
    """Any per-step choice between two exact samplers is exact: paths follow Eq. (prob)."""
    g = triangle_graph()
    lg = oracle.Logic(**logic)
    n = 60000
    for start in (0, 4):
        probs = exact.path_distribution(g, lg, start, 3)
        assert_chisq(lambda s: chisq_pvalue(_walk_counts(g, lg, oracle.Plan(d_lo=3, lanes=2), strategy, start, 3, n,
                                                         seed=s)[0], probs, n), 51 + start, start)


def test_selection_policy_ratios():
    """The fair coin picks eRJS for about half the steps; the degree policy picks eRJS for
    exactly the steps taken from vertices of degree >= d_lo."""
    g = synth.rmat(12, 8 << 12, seed=2)
    og = oracle.Graph(g)
    lg = oracle.Logic(**N2V)
    st = np.arange(g["nv"], dtype=np.int32)
    r = oracle.walk(og, lg, oracle.Plan(rjs_cap=1 << 20), oracle.RANDOM_SELECT, st, 20, 3, diagnostics=False)
    n = r.counters["steps"]
    assert abs(r.counters["rjs_steps"] / n - 0.5) < 5 * math.sqrt(0.25 / n)
    pl = oracle.Plan(d_lo=40, rjs_cap=1 << 20)
    r = oracle.walk(og, lg, pl, oracle.DEGREE_SELECT, st, 20, 3)
    deg = np.diff(g["row_ptr"])
    taken = np.arange(20)[None, :] < r.lengths[:, None]
    from_high = (deg[np.where(taken, r.paths[:, :-1], 0)] >= 40) & taken
    assert r.counters["rjs_steps"] == int(from_high.sum())
    assert (r.kinds[taken] == np.where(from_high[taken], 1, 0)).all()


# ------------------------------------------------------------------ closed form / invariants
def test_stationary_visits_proportional_to_degree():
    """p = q = 1, h = 1 on a connected non-bipartite graph: visits -> deg / 2|E|."""
    g = triangle_graph()
    g = synth.csr_from_edges(6, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3), (3, 4), (2, 4), (4, 5), (0, 5)])
    lg = oracle.Logic(kind=oracle.NODE2VEC, weighted=False, p=1.0, q=1.0)
    og = oracle.Graph(g)
    r = oracle.walk(og, lg, oracle.Plan(rho=1.0, lanes=2), oracle.AUTO, np.zeros(400, np.int32), 2000, 9,
                    diagnostics=False)
    visits = np.bincount(r.paths[:, 200:].ravel(), minlength=6) / r.paths[:, 200:].size
    deg = np.diff(g["row_ptr"]) / g["row_ptr"][-1]
    np.testing.assert_allclose(visits, deg, atol=0.01)


def _check_invariants(g, lg, paths, lengths, L):
    rp, col = g["row_ptr"], g["col"]
    for i in range(paths.shape[0]):
        n = int(lengths[i])
        prev = -1
        for j in range(n):
            cur, nxt = int(paths[i, j]), int(paths[i, j + 1])
            row = col[rp[cur]:rp[cur + 1]]
            k = int(np.searchsorted(row, nxt))
            assert k < row.size and row[k] == nxt, "step must land on a neighbour"
            assert exact.transition_weight(g, lg, j, prev, int(rp[cur]) + k) > 0, "weight must be positive"
            prev = cur
        assert (paths[i, n + 1:] == -1).all()
        if n < L:  # ended early only when no neighbour has positive weight
            assert exact.transition(g, lg, n, prev, int(paths[i, n])) == {}


@pytest.mark.parametrize("strategy", [oracle.AUTO, oracle.RVS_ONLY, oracle.RJS_ONLY])
def test_invariants_rmat(strategy):
    g = synth.rmat(9, 8 << 9, seed=2, nlabels=5)
    og = oracle.Graph(g)
    starts = synth.uniform_starts(g["nv"], 300, 4)
    for lg in (oracle.Logic(**N2V), oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2, 3, 4))):
        r = oracle.walk(og, lg, oracle.Plan(rho=4.0, rjs_cap=64), strategy, starts, 12, 42)
        _check_invariants(g, lg, r.paths, r.lengths, 12)
        if lg.kind == oracle.METAPATH:
            rp, col, lab = g["row_ptr"], g["col"], g["label"]
            for i in range(len(starts)):
                for j in range(int(r.lengths[i])):
                    a, b = int(r.paths[i, j]), int(r.paths[i, j + 1])
                    k = rp[a] + np.searchsorted(col[rp[a]:rp[a + 1]], b)
                    assert lab[k] == lg.schema[j % 5]


def test_determinism_and_walker_ids():
    """The stream depends on (seed, walker id, step, draw) only, not on the batch."""
    g = synth.rmat(10, 8 << 10, seed=2)
    og = oracle.Graph(g)
    lg = oracle.Logic(**N2V)
    starts = synth.uniform_starts(g["nv"], 500, 1)
    full = oracle.walk(og, lg, oracle.Plan(), oracle.AUTO, starts, 10, 42, diagnostics=False)
    sub = np.arange(100, 500, 7)
    part = oracle.walk(og, lg, oracle.Plan(), oracle.AUTO, starts[sub], 10, 42, walker_ids=sub, diagnostics=False)
    np.testing.assert_array_equal(full.paths[sub], part.paths)
    again = oracle.walk(og, lg, oracle.Plan(), oracle.AUTO, starts, 10, 42, diagnostics=False, nthreads=1)
    np.testing.assert_array_equal(full.paths, again.paths)


# ------------------------------------------------------------------ cost model, sum estimate, bytes
def _kind(g, lg, plan, j, prev, cur, strategy=oracle.AUTO):
    """eRJS (1, or 2 when capped) or eRVS (0) at one hand-computed state."""
    k = oracle.step_info(oracle.Graph(g), lg, plan, strategy, 3, 0, j, prev, cur)["kind"]
    return {0: "rvs", 1: "rjs", 2: "rjs"}[k]


# (state, logic, B, S^) by hand from Section 4.1 Eq. (runtime) and Section 4.2 Eq.
# (sum_estimation): B = max(w) * h_MAX[v], S^ = mean over the logic's return values of w,
# times h_SUM[v].  The paper's plan (uniform proposals, bound max(w) * h_MAX) compares rho * B
# with S^ and takes eRJS only when rho * B < S^ (a tie goes to eRVS).
def _selector_cases():
    tri, tri_l = triangle_graph(), triangle_graph(labels=True)
    return [
        # Node2Vec a = 2, b = 1/2 at prev = 0, cur = 1: N(1) = {0, 2, 3}, h = 1, 3, 4, so
        # h_MAX = 4, h_SUM = 8; w in {1/2, 1, 2}: B = 2 * 4 = 8, mean (1/2 + 1 + 2) / 3 = 7/6,
        # S^ = fl(fl(7/6) * 8)
        ("node2vec", tri, oracle.Logic(**N2V), 1, 0, 1, 8.0,
         float(np.float32(np.float32(np.float32(np.float32(0.5) + np.float32(1)) + np.float32(2)) / np.float32(3))
               * np.float32(8))),
        # MetaPath: w in {1, 0}, B = 1 * h_MAX, S^ = (1 + 0) / 2 * h_SUM; N(2) has h = 2, 3, 1, 3
        ("metapath", tri_l, oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2)), 1, 0, 2, 3.0, 4.5),
        # second-order PageRank gamma = 1/4 at prev = 2 (d 4), cur = 1 (d 3): max_d = 4,
        # w in {5/4, 1}: B = 5/4 * 4 = 5, S^ = (5/4 + 1) / 2 * 8 = 9
        ("2ndpr", tri, oracle.Logic(**PR2), 1, 2, 1, 5.0, 9.0),
        # unweighted Node2Vec a = b = 1: every w = 1, h = 1: B = 1, S^ = d(1) = 3
        ("unweighted", tri, oracle.Logic(kind=oracle.NODE2VEC, weighted=False, p=1.0, q=1.0), 1, 0, 1, 1.0, 3.0),
        # first step (no previous vertex): w = 1 for every logic with one: B = h_MAX = 4, S^ = h_SUM = 8
        ("first_step", tri, oracle.Logic(**N2V), 0, -1, 1, 4.0, 8.0),
    ]


def _pin_selector():
    for name, g, lg, j, prev, cur, B, S in _selector_cases():
        B32, S32 = np.float32(B), np.float32(S)
        rho_tie = np.float32(S32 / B32)
        assert np.float32(rho_tie * B32) == S32, name  # an exact float32 tie
        for rho, want in ((rho_tie * np.float32(0.98), "rjs"), (rho_tie, "rvs"), (rho_tie * np.float32(1.02), "rvs")):
            got = _kind(g, lg, oracle.Plan(rho=float(rho)), j, prev, cur)
            assert got == want, (name, float(rho), float(rho * B32), S, got)
        # the degree gate: below d_lo every step is eRVS, whatever the cost model says
        deg = int(g["row_ptr"][cur + 1] - g["row_ptr"][cur])
        assert _kind(g, lg, oracle.Plan(rho=float(rho_tie) * 0.5, d_lo=deg + 1), j, prev, cur) == "rvs", name
        assert _kind(g, lg, oracle.Plan(rho=float(rho_tie) * 0.5, d_lo=deg), j, prev, cur) == "rjs", name


def test_cost_model_selector_and_sum_estimate():
    """Which kernel AUTO picks at hand-computed states on both sides of rho * B = S^ (and at
    the exact tie, which goes to eRVS): pins the bound B, the sum estimate S^ (its mean over
    the logic's return values: Node2Vec's three, MetaPath's two, second-order PageRank's two)
    and the direction of Eq. (runtime)."""
    _pin_selector()


def _directed(nv, rows, h=None):
    """CSR from {v: [sorted neighbours]} (directed: the byte pins need states whose
    membership outcomes are fixed)."""
    rp = np.zeros(nv + 1, np.int64)
    col = []
    for v in range(nv):
        col += rows.get(v, [])
        rp[v + 1] = len(col)
    g = {"nv": nv, "ne": len(col), "row_ptr": rp, "col": np.array(col, np.int32), "h": None, "label": None}
    if h is not None:
        g["h"] = np.full(len(col), h, np.float32)
    return g


def _pin_bytes():
    """Hand-counted algorithmic bytes of single steps (the byte model of the measurement
    plan: 16 B for the row pointer pair, 4 B of h_MAX and 4 B of h_SUM where the step reads
    them, 4 B col + 4 B h (+1 B label) per scanned or proposed edge, on every eRJS trial of a
    board whose acceptance depends on u in N(v') a binary search of N(v') in 4 B probes
    (ceil(log2(d(v') + 1)) of them), for an eRVS step the cheaper of staging N(v') and one such
    search per scanned edge, the h-proportional proposal's alias col, alias h and threshold
    (12 B), a member-region trial's neighbour of v' (4 B), a binary search of v's row and
    h(v, x) (4 B when weighted), and 4 B start + 4 B per path slot + 4 B length per walk)."""
    # v = 0 with N(0) = {2}; v' = 1 with N(1) = {2, 3, 4, 5, 6} (5 entries: ceil(log2 6) = 3
    # probes); Node2Vec a = 1, b = 2^30: w = 1 on N(v'), ~1e-9 elsewhere, so every proposal's
    # accept test is left open by the bounds of w and needs the membership test.
    g = _directed(8, {0: [2], 1: [2, 3, 4, 5, 6], 7: [3]})
    n2v = oracle.Logic(kind=oracle.NODE2VEC, weighted=False, p=1.0, q=float(2 ** 30))
    og = oracle.Graph(g)

    def b(lg, plan, strategy, j, prev, cur, graph=og):
        return oracle.step_info(graph, lg, plan, strategy, 3, 0, j, prev, cur)["bytes"]

    # one eRJS trial (proposes 2, a member): 16 + 4 (col) + 3 probes * 4 B
    assert b(n2v, oracle.Plan(), oracle.RJS_ONLY, 1, 1, 0) == 16 + 4 + 12
    # v = 7 with N(7) = {3}, v' = 1: 3 is a member, but now test a non-member: v' = 0 with N(0) = {2}
    # (one probe): every trial rejects, so rjs_cap = 3 trials, then eRVS scans 1 entry and
    # tests it (min(4 * d(v'), 4 * deg * probes) = min(4, 4) bytes)
    assert b(n2v, oracle.Plan(rjs_cap=3), oracle.RJS_ONLY, 1, 0, 7) == 16 + 3 * (4 + 4 * 1) + (4 + 4)
    # the search is charged on every trial, also one whose accept test the weight bounds
    # already decide (a = b = 1: every neighbour weighs 1)
    flat = oracle.Logic(kind=oracle.NODE2VEC, weighted=False, p=1.0, q=1.0)
    assert b(flat, oracle.Plan(), oracle.RJS_ONLY, 1, 1, 0) == 16 + 4 + 12
    # the first step has no membership at all
    assert b(n2v, oracle.Plan(), oracle.RJS_ONLY, 0, -1, 0) == 16 + 4
    # eRVS: d(v) = 5 entries of 4 B; N(v') staged (4 * d(v') = 4) against 5 searches of 1 probe
    assert b(n2v, oracle.Plan(), oracle.RVS_ONLY, 1, 0, 1) == 16 + 5 * 4 + min(4 * 1, 4 * 5 * 1)
    # ... and with N(v') = 5 entries against a 1-entry row: one search of 3 probes (12) < staging (20)
    assert b(n2v, oracle.Plan(), oracle.RVS_ONLY, 1, 1, 0) == 16 + 1 * 4 + min(4 * 5, 4 * 1 * 3)
    # weighted: 4 B of h per edge, and h_MAX (eRJS only) or h_MAX + h_SUM (the cost model)
    gw = _directed(8, {0: [2], 1: [2, 3, 4, 5, 6], 7: [3]}, h=2.0)
    ogw = oracle.Graph(gw)
    n2vw = oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=1.0, q=float(2 ** 30))
    assert b(n2vw, oracle.Plan(), oracle.RJS_ONLY, 1, 1, 0, ogw) == 16 + 4 + (4 + 4) + 12
    assert b(n2vw, oracle.Plan(rho=1e-6), oracle.AUTO, 1, 1, 0, ogw) == 16 + 8 + (4 + 4) + 12
    # h-proportional proposal: its record adds the alias col, alias h and threshold (12 B)
    assert b(n2vw, oracle.Plan(proposal=1), oracle.RJS_ONLY, 1, 1, 0, ogw) == 16 + 4 + (4 + 4 + 12) + 12
    # member board (second-order PageRank, gamma = 1: only members of N(v') weigh anything,
    # so every trial is a member-region trial): v = 0 with N(0) = {1, 2}, v' = 1 with
    # N(1) = {2}: the trial reads x = 2 (4 B) and looks (0, 2) up: a search of the 2-entry row
    # (ceil(log2 3) = 2 probes); it is kept, h = 1 = h_MAX
    gm = _directed(3, {0: [1, 2], 1: [2]})
    ogm = oracle.Graph(gm)
    pr1 = oracle.Logic(kind=oracle.SECOND_PR, weighted=False, gamma=1.0)
    assert b(pr1, oracle.Plan(bound=2), oracle.RJS_ONLY, 1, 1, 0, ogm) == 16 + 4 + 4 * 2
    # ... weighted (h = 2 everywhere): h_MAX (4 B), and h(0, 2) with the member trial
    gmw = _directed(3, {0: [1, 2], 1: [2]}, h=2.0)
    pr1w = oracle.Logic(kind=oracle.SECOND_PR, weighted=True, gamma=1.0)
    assert b(pr1w, oracle.Plan(bound=2), oracle.RJS_ONLY, 1, 1, 0, oracle.Graph(gmw)) == 16 + 4 + (4 + 4 * 2 + 4)
    # label-conditioned MetaPath proposal: the group's two positions (8 B), then one trial:
    # col, h and label (9 B) and the alias slot's col, h and threshold (12 B)
    gl = synth.csr_from_edges(3, [(0, 1), (0, 2)], h=[2.0, 3.0], label=[0, 1])
    mpl = oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(1,))
    assert b(mpl, oracle.Plan(proposal=2), oracle.RJS_ONLY, 0, -1, 0, oracle.Graph(gl)) == 16 + 8 + 9 + 12
    # a walk's own I/O: a start at an isolated vertex reads its row pointers and ends:
    # 4 (start) + 4 * (L + 1) (path row) + 4 (length) + 16
    r = oracle.walk(og, n2v, oracle.Plan(), oracle.AUTO, np.array([5], np.int32), 7, 1)
    assert r.lengths[0] == 0 and r.counters["alg_bytes"] == 4 + 4 * 8 + 4 + 16


def test_algorithmic_bytes_hand_counted():
    _pin_bytes()


# ------------------------------------------------------------------ planted mistakes
MUTANTS = {
    1: "Node2Vec return weight uses 1/q",
    2: "jump key not conditioned on beating the threshold",
    3: "skip sum not reset after a jump",
    4: "eRJS never proposes the last neighbour",
    5: "eRJS bound without h_MAX",
    6: "split bound's extra column is the whole return weight",
    7: "second-order PageRank divides gamma by d(v) instead of d(v')",
    8: "alias tables never take the alias",
    9: "member region keeps a member without its h test",
    10: "sum estimate averages Node2Vec over 2 branches instead of 3",
    11: "cost model's choice inverted",
    12: "row pointer pair charged 8 bytes instead of 16",
    13: "label groups proposed uniformly, ignoring h",
    14: "shared eRVS threshold rescales the skip by the inverted ratio",
    15: "shared eRVS threshold taken without rescaling the skip",
}
# planted mistakes caught by a pin of their own: hand-computed states (10-13), or the
# hub-row chi-square of the shared eRVS threshold (14, 15), where the triangle graph's
# rows are too short for the scan to pass a shared threshold often
OWN_PINS = {10: "_pin_selector", 11: "_pin_selector", 12: "_pin_bytes", 13: "_pin_label_groups",
            14: "_pin_rvs_share", 15: "_pin_rvs_share"}


def _pin_label_groups():
    test_label_groups_realise_h("pareto1")


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    d = tmp_path_factory.mktemp("mutants")
    return {k: oracle.build_variant(str(d / f"liboracle_m{k}.so"), {"OG_MUTANT": k}) for k in MUTANTS}


@pytest.mark.parametrize("mut", sorted(MUTANTS), ids=[MUTANTS[k] for k in sorted(MUTANTS)])
def test_planted_mistake_is_caught(mut, mutant_libs):
    if mut in OWN_PINS:
        with oracle.use_library(mutant_libs[mut]):
            with pytest.raises(AssertionError):
                globals()[OWN_PINS[mut]]()
        return
    g = triangle_graph(labels=True)
    caught = []
    with oracle.use_library(mutant_libs[mut]):
        for name, logic, strategy, plan in (("rvs_P2", N2V, oracle.RVS_ONLY, oracle.Plan(lanes=2)),
                                            ("rvs_P1", N2V, oracle.RVS_ONLY, oracle.Plan(lanes=1)),
                                            ("rjs", N2V, oracle.RJS_ONLY, oracle.Plan()),
                                            ("rjs_split", N2V_RET, oracle.RJS_ONLY, oracle.Plan(bound=1)),
                                            ("rjs_2ndpr", PR2, oracle.RJS_ONLY, oracle.Plan()),
                                            ("rvs_2ndpr", PR2, oracle.RVS_ONLY, oracle.Plan(lanes=2)),
                                            ("rjs_hprop", N2V, oracle.RJS_ONLY, oracle.Plan(proposal=1)),
                                            ("rjs_member", PR2, oracle.RJS_ONLY, oracle.Plan(bound=2)),
                                            ("rjs_label", MP_L, oracle.RJS_ONLY, oracle.Plan(proposal=2))):
            lg = oracle.Logic(**logic)
            n = 60000
            counts, _ = _walk_counts(g, lg, plan, strategy, 0, 3, n, seed=7)
            probs = exact.path_distribution(g, lg, 0, 3)
            caught.append(chisq_pvalue(counts, probs, n) < P_BAD)
    assert any(caught), MUTANTS[mut]


# ------------------------------------------------------------------ 8-bit property weights
def test_dequantize_h8_exact():
    """h = h_scale * code rounded once to float32: the product of an 8-bit and a 24-bit
    integer significand is exact in double, so rounding that double to float32 is the
    correctly rounded product."""
    codes = np.arange(256, dtype=np.uint8)
    for scale in (np.float32(10.0 / 255.0), np.float32(1.0), np.float32(3e-5), np.float32(7.0),
                  np.float32(1e30)):
        got = oracle.dequantize_h8(codes, scale)
        want = (codes.astype(np.float64) * np.float64(scale)).astype(np.float32)
        np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))


def _q8(g):
    """The graph with its weights as 8-bit codes, and the float graph of the same weights."""
    codes, scale = synth.quantize_u8(g["h"])
    gq = dict(g, h=None, h8=codes, h_scale=scale)
    gf = dict(g, h=(codes.astype(np.float64) * np.float64(scale)).astype(np.float32))
    return gq, gf


@pytest.mark.parametrize("strategy", [oracle.RVS_ONLY, oracle.RJS_ONLY, oracle.AUTO], ids=["rvs", "rjs", "auto"])
def test_h8_walks_equal_float_walks(strategy):
    """A graph given as 8-bit codes walks exactly like the float graph of the dequantised
    weights; only the algorithmic bytes differ: 3 bytes less per scanned or proposed
    edge."""
    g = synth.rmat(8, 8 << 8, seed=3)
    g["h"], _ = synth.edge_props(g["row_ptr"], g["col"], 5)
    gq, gf = _q8(g)
    st = synth.all_vertices(g["nv"])
    lg = oracle.Logic(**N2V)
    pl = oracle.Plan(rho=1.0, rjs_cap=1 << 20)
    a = oracle.walk(oracle.Graph(gq), lg, pl, strategy, st, 12, 21)
    b = oracle.walk(oracle.Graph(gf), lg, pl, strategy, st, 12, 21)
    np.testing.assert_array_equal(a.paths, b.paths)
    for k in a.counters:
        if k != "alg_bytes":
            assert a.counters[k] == b.counters[k], k
    # items moved: every eRVS step scans deg(v) edges, every eRJS trial reads one edge
    deg = np.diff(g["row_ptr"])
    items = 0
    for p, n in zip(a.paths, a.lengths):
        for j in range(n):
            items += 0 if strategy == oracle.RJS_ONLY else int(deg[p[j]])
    if strategy == oracle.RJS_ONLY:
        items = int(a.counters["rjs_trials"])
    if strategy != oracle.AUTO:
        assert b.counters["alg_bytes"] - a.counters["alg_bytes"] == 3 * items
    else:
        assert b.counters["alg_bytes"] > a.counters["alg_bytes"]


def test_h8_chisquare():
    """Paths on the triangle graph with 8-bit weights follow the exact distribution of the
    dequantised weights."""
    g = triangle_graph()
    codes = np.array([3, 200, 17, 255, 1, 90, 44, 128, 64], np.uint8)
    g8 = synth.csr_from_edges(7, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3), (3, 4), (2, 4), (4, 5), (0, 5)],
                              h=list(range(9)))
    # the helper stores h per CSR entry from the edge list: map each entry to its code
    idx = g8["h"].astype(np.int64)
    scale = np.float32(0.37)
    gq = dict(g, h=None, h8=codes[idx], h_scale=scale)
    gf = dict(g, h=(codes[idx].astype(np.float64) * np.float64(scale)).astype(np.float32))
    lg = oracle.Logic(**N2V)
    n = 60000
    probs = exact.path_distribution(gf, lg, 0, 3)
    for strategy, plan in ((oracle.RJS_ONLY, oracle.Plan()), (oracle.RVS_ONLY, oracle.Plan(lanes=2)),
                           (oracle.RJS_ONLY, oracle.Plan(proposal=1, bound=2))):
        assert_chisq(lambda s: chisq_pvalue(_walk_counts(gq, lg, plan, strategy, 0, 3, n, seed=s)[0], probs, n), 5,
                     (strategy, plan.bound))
