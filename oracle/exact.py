"""Exact transition and path probabilities of a dynamic random walk.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The plain definition of FlexiWalker (arXiv 2512.00705), Section 2.1, written out in
rational arithmetic:

* transition weight w~(v, u) = w(v, u) * h(v, u), probability
  p(u) = w~(v, u) / sum_{t in N(v)} w~(v, t)  (Eq. prob);
* Node2Vec (Eq. node2vec): w = 1/a if u is the previous vertex (dist 0), 1 if u is a
  neighbour of the previous vertex (dist 1), 1/b otherwise (dist 2); a, b are called
  p, q here.  The first step has no previous vertex and uses w = 1;
* MetaPath: w = 1 when the edge label equals the schema label of the current step
  (schema repeated along the walk), else 0;
* second-order PageRank (Eq. 2ndpr): with max_d = max(d(v), d(v')),
  w = ((1 - gamma)/d(v) + gamma/d(v')) * max_d if u is a neighbour of v' (dist 1),
  else ((1 - gamma)/d(v)) * max_d; the first step has no v' and uses w = 1.

A walk ends early when the current vertex has no neighbour of positive weight.
Float inputs (p, q, h) are converted to fractions exactly.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

NODE2VEC, METAPATH, SECOND_PR = 1, 2, 3


def _row(g, v):
    return range(int(g["row_ptr"][v]), int(g["row_ptr"][v + 1]))


def workload_weight(g, logic, j: int, prev: int, k: int) -> Fraction:
    """w(v, u) for the edge at CSR position k (u = col[k]) at step j."""
    u = int(g["col"][k])
    if logic.kind == NODE2VEC:
        if j == 0:
            return Fraction(1)
        if u == prev:
            return 1 / Fraction(float(logic.p))
        if any(int(g["col"][t]) == u for t in _row(g, prev)):  # plain scan of N(prev)
            return Fraction(1)
        return 1 / Fraction(float(logic.q))
    if logic.kind == METAPATH:
        return Fraction(1) if int(g["label"][k]) == logic.schema[j % len(logic.schema)] else Fraction(0)
    if logic.kind == SECOND_PR:
        if j == 0:
            return Fraction(1)
        cur = int(np.searchsorted(g["row_ptr"], k, side="right")) - 1  # the row holding position k
        dv, dvp = len(_row(g, cur)), len(_row(g, prev))
        gamma = Fraction(float(logic.gamma))
        max_d = max(dv, dvp)
        if u != prev and any(int(g["col"][t]) == u for t in _row(g, prev)):
            return ((1 - gamma) / dv + gamma / dvp) * max_d
        return (1 - gamma) / dv * max_d
    raise ValueError(logic.kind)


def transition_weight(g, logic, j: int, prev: int, k: int) -> Fraction:
    w = workload_weight(g, logic, j, prev, k)
    if logic.weighted and g.get("h") is not None:
        return w * Fraction(float(g["h"][k]))
    return w


def transition(g, logic, j: int, prev: int, cur: int) -> dict:
    """{next vertex: exact probability}; empty when the walk ends at this state."""
    ws = {int(g["col"][k]): transition_weight(g, logic, j, prev, k) for k in _row(g, cur)}
    total = sum(ws.values(), Fraction(0))
    if total == 0:
        return {}
    return {u: w / total for u, w in ws.items() if w > 0}


def path_distribution(g, logic, start: int, L: int) -> dict:
    """Brute-force enumeration of every walk of at most L steps from ``start``.

    Keys are (L+1)-tuples padded with -1 after an early end, values exact
    probabilities (they sum to 1).
    """
    out: dict = {}

    def rec(path, prob, prev, cur, j):
        if j == L:
            out[tuple(path)] = out.get(tuple(path), 0) + prob
            return
        t = transition(g, logic, j, prev, cur)
        if not t:
            key = tuple(path + [-1] * (L - j))
            out[key] = out.get(key, 0) + prob
            return
        for u, pu in t.items():
            rec(path + [u], prob * pu, cur, u, j + 1)

    rec([int(start)], Fraction(1), -1, int(start), 0)
    return out


def first_order_matrix(g, weighted: bool = True) -> np.ndarray:
    """Row-stochastic matrix of the static walk p(u|v) = h(v,u) / sum h (float64)."""
    n = int(g["nv"])
    P = np.zeros((n, n))
    for v in range(n):
        for k in _row(g, v):
            P[v, int(g["col"][k])] += float(g["h"][k]) if (weighted and g.get("h") is not None) else 1.0
        s = P[v].sum()
        if s > 0:
            P[v] /= s
    return P
