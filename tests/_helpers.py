"""Shared test fixtures: tiny graphs and a chi-square helper."""
from __future__ import annotations

import numpy as np
from scipy import stats

import synth


def chisq_pvalue(counts: dict, probs: dict, n: int, min_expected: float = 5.0) -> float:
    """Pearson chi-square p-value of observed counts against exact probabilities.

    Categories observed with probability zero give p = 0.  Categories with expected
    count below ``min_expected`` are pooled (smallest first) into one bin.
    """
    for k, c in counts.items():
        if c > 0 and float(probs.get(k, 0)) == 0.0:
            return 0.0
    keys = sorted(probs, key=lambda k: float(probs[k]))
    exp = np.array([n * float(probs[k]) for k in keys])
    obs = np.array([counts.get(k, 0) for k in keys], dtype=float)
    bins_e, bins_o = [], []
    acc_e = acc_o = 0.0
    for e, o in zip(exp, obs):
        acc_e += e
        acc_o += o
        if acc_e >= min_expected:
            bins_e.append(acc_e)
            bins_o.append(acc_o)
            acc_e = acc_o = 0.0
    if acc_e > 0:
        if bins_e:
            bins_e[-1] += acc_e
            bins_o[-1] += acc_o
        else:
            bins_e.append(acc_e)
            bins_o.append(acc_o)
    if len(bins_e) < 2:
        return 1.0
    e, o = np.array(bins_e), np.array(bins_o)
    stat = float(((o - e) ** 2 / e).sum())
    return float(stats.chi2.sf(stat, len(e) - 1))


def path_counts(paths: np.ndarray) -> dict:
    uniq, cnt = np.unique(paths, axis=0, return_counts=True)
    return {tuple(int(x) for x in u): int(c) for u, c in zip(uniq, cnt)}


def worked_example_graph() -> dict:
    """v0 with neighbours v1..v4 and property weights 3, 2, 4, 1 (star)."""
    return synth.csr_from_edges(5, [(0, 1), (0, 2), (0, 3), (0, 4)], h=[3, 2, 4, 1])


def triangle_graph(labels: bool = False) -> dict:
    """Seven vertices with triangles, a pendant vertex and an isolated vertex.

    Integer weights keep every float32 product exact.  Rows hold all three Node2Vec
    cases (return, common neighbour, two hops).
    """
    edges = [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3), (3, 4), (2, 4), (4, 5), (0, 5)]
    h = [1, 2, 3, 4, 1, 2, 3, 1, 2]
    lab = [0, 1, 2, 0, 1, 2, 0, 1, 2] if labels else None
    g = synth.csr_from_edges(7, edges, h=h, label=lab)
    # vertex 6 is isolated
    return g


def hub_ring_graph(n_leaves: int = 600, seed: int = 3) -> dict:
    """Hub 0 joined to leaves 1..n; leaves form a ring.  Hashed weights in [1, 10)."""
    edges = [(0, i) for i in range(1, n_leaves + 1)]
    edges += [(i, i % n_leaves + 1) for i in range(1, n_leaves + 1)]
    g = synth.csr_from_edges(n_leaves + 1, edges)
    h, _ = synth.edge_props(g["row_ptr"], g["col"], seed)
    g["h"] = h
    return g


P_MIN = 0.01          # chi-square acceptance level of the parity target (p > 0.01)
RETEST_OFFSET = 1_000_003


def assert_chisq(pvalue_of_seed, seed: int, label: str = "") -> float:
    """Chi-square acceptance at p > 0.01 with one declared retest.

    ``pvalue_of_seed(s)`` runs the sampler with seed ``s`` and returns the p-value of its
    counts against the exact probabilities.  The test passes when p > 0.01 at ``seed``;
    otherwise one retest on the independent seed ``seed + RETEST_OFFSET`` must give
    p > 0.01.  Fixed seeds make every run deterministic.  A correct sampler fails both with
    probability 1e-4; a biased one gives small p at both seeds.  A retest is printed, so the
    test log shows which cases needed one.
    """
    p0 = float(pvalue_of_seed(seed))
    if p0 > P_MIN:
        return p0
    p1 = float(pvalue_of_seed(seed + RETEST_OFFSET))
    print(f"chi-square retest {label}: p = {p0:.3g} at seed {seed}, p = {p1:.3g} at seed {seed + RETEST_OFFSET}")
    assert p1 > P_MIN, (label, p0, p1)
    return p1
