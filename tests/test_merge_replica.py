"""Host replica of the eRVS merge's control flow (the wave-wide membership test u in N(prev)).

The eRVS scan takes the items of a sorted row 64 at a time (one per lane, a prefix of the
lanes holding items in the last round) and decides for each whether it lies in N(prev),
also sorted, by walking a cursor through N(prev) in blocks of 64 (Section 3.2's scan with
the Node2Vec weight of Eq. (node2vec), whose middle case is that membership).  Two forms
run on the device: the bisection of each lane's item in the block, and, in the eRVS-only
kernel variant, the broadcast of the few block entries that lie between the round's
smallest and largest item (a bisection when there are more than 8), the cursor moving
past every entry up to the largest item.  This replica restates both loops in plain Python
and checks them against set membership over whole scans: dense and sparse N(prev), empty
N(prev), N(prev) entirely below or above the row, entries equal to a round's first or
last item, ragged last rounds (invalid lanes hold item 0 while vertex 0 is in N(prev)),
and rounds whose range covers several blocks.
"""
from __future__ import annotations

import numpy as np
import pytest

W = 64
BIG = 2**31 - 1


def _block(nprev, lo):
    return [int(nprev[lo + l]) if lo + l < len(nprev) else BIG for l in range(W)]


def merge_bisect(nprev, items, valid, lo):
    """The bisection form: (found per lane, new cursor)."""
    vm = [l for l in range(W) if valid[l]]
    if not vm:
        return [False] * W, lo
    umax = items[vm[-1]]
    found = [False] * W
    done = [not valid[l] for l in range(W)]
    first = True
    while True:
        v = _block(nprev, lo)
        if first and umax < v[0]:
            return [False] * W, lo
        first = False
        cs = []
        for l in range(W):
            u, c = items[l], 0
            for s in (32, 16, 8, 4, 2, 1):
                if v[c + s - 1] < u:
                    c += s
            cs.append(c)
            if not done[l]:
                found[l] = c < W and v[c & (W - 1)] == u
                done[l] = u <= v[W - 1]
        if all(done):
            break
        lo += W
    return found, lo + cs[W - 1]


def merge_broadcast(nprev, items, valid, lo, bcast=8):
    """The eRVS-only variant's form: (found per lane, new cursor)."""
    vm = [l for l in range(W) if valid[l]]
    if not vm:
        return [False] * W, lo
    umin, umax = items[vm[0]], items[vm[-1]]
    v = _block(nprev, lo)
    if umax < v[0]:
        return [False] * W, lo
    found = [False] * W
    while True:
        inr = [l for l in range(W) if umin <= v[l] <= umax]
        if len(inr) <= bcast:
            for b in inr:
                e = v[b]
                found = [found[l] or items[l] == e for l in range(W)]
        else:
            for l in range(W):
                u, c = items[l], 0
                for s in (32, 16, 8, 4, 2, 1):
                    if v[c + s - 1] < u:
                        c += s
                found[l] = found[l] or (c < W and v[c & (W - 1)] == u)
        le = [l for l in range(W) if v[l] <= umax]
        assert le == list(range(len(le))), "entries up to the largest item form a prefix"
        if len(le) < W:
            lo += len(le)
            break
        lo += W
        v = _block(nprev, lo)
    return [found[l] and valid[l] for l in range(W)], lo


def scan(merge, row, nprev, **kw):
    """Membership of every row entry, the row scanned in rounds of 64 with one cursor."""
    out, lo = [], 0
    for r0 in range(0, len(row), W):
        items = [int(row[r0 + l]) if r0 + l < len(row) else 0 for l in range(W)]
        valid = [r0 + l < len(row) for l in range(W)]
        f, lo2 = merge(nprev, items, valid, lo, **kw)
        assert lo2 >= lo
        # the cursor never passes an entry larger than this round's largest item
        if any(valid):
            umax = max(items[l] for l in range(W) if valid[l])
            assert all(x <= umax for x in nprev[lo:lo2])
        lo = lo2
        out += f[:sum(valid)]
    return out


def _sorted_sample(rng, universe, k):
    return np.sort(rng.choice(universe, size=min(k, universe), replace=False)).astype(np.int64)


CASES = [  # (row length, N(prev) length, universe)
    (1, 0, 10), (5, 3, 10), (64, 64, 200), (65, 1, 100), (3000, 200, 100000), (3000, 2500, 20000),
    (2770, 2576, 10000), (200, 6000, 8000), (130, 5000, 5200), (700, 700, 700), (63, 40000, 50000),
    (4000, 30, 4100),
]


@pytest.mark.parametrize("bcast", [8, 0, 64])
@pytest.mark.parametrize("case", CASES, ids=[f"{a}x{b}" for a, b, _ in CASES])
def test_merge_forms_equal_membership(case, bcast):
    n_row, n_prev, universe = case
    rng = np.random.default_rng(n_row * 7 + n_prev)
    for rep in range(3):
        row = _sorted_sample(rng, universe, n_row)
        nprev = _sorted_sample(rng, universe, n_prev)
        if rep == 1 and n_prev:
            nprev[0] = 0  # vertex 0 in N(prev): invalid lanes carry item 0
        if rep == 2 and n_prev and n_row > 64:
            # entries equal to a round's first and last items, and N(prev) ending inside a round
            nprev = np.unique(np.concatenate([nprev[: n_prev // 2], row[[0, 63, 64]]]))
        want = [bool(x) for x in np.isin(row, nprev)]
        assert scan(merge_bisect, row, nprev) == want
        assert scan(merge_broadcast, row, nprev, bcast=bcast) == want


def test_merge_extremes():
    """N(prev) entirely below or above the row, empty, and identical to it."""
    row = np.arange(1000, 1300, dtype=np.int64)
    for nprev in (np.arange(0, 500), np.arange(2000, 2600), np.zeros(0, np.int64), row.copy()):
        want = [bool(x) for x in np.isin(row, nprev)]
        assert scan(merge_bisect, row, nprev) == want
        assert scan(merge_broadcast, row, nprev) == want
