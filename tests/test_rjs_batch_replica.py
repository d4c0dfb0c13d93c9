"""Host replica of the eRJS proposal batch's control flow, depths 1 to 5.

The walk kernel draws the proposals of trials t, t+1, ..., t+K-1 of a lane together
(K = the batch depth), stops drawing after a proposal whose acceptance its own uniforms
already decide (a "sure" trial), then decides the slots in trial order, shifting the
batch down one slot per trial, and falls back to eRVS once the trial count reaches the
cap (Section 3.3: the first accepted proposal is the sample; a capped step is re-sampled
exactly).  The definition is the sequential loop: the first t < cap with acc(t), else a
fall-back after cap trials.  This replica restates the kernel's loop (fill, sure-skip,
decide with the shift, cap test after each trial) in plain Python and checks it against
the sequential loop on random acceptance patterns, for every depth 1..5 and every cap
1..13, so that batch boundaries fall before, on and after the cap and the sure trial.
"""
from __future__ import annotations

import numpy as np
import pytest

EMPTY = None


def sequential(acc, cap):
    """(outcome, trials): ('acc', t) at the first accepted trial t < cap, else ('rvs', cap)."""
    for t in range(cap):
        if acc[t]:
            return "acc", t + 1
    return "rvs", cap


def batched(acc, sure, cap, depth):
    """The kernel's loop: per batch, fill `depth` slots (trial numbers) unless a sure trial
    came first, then decide slot 0 up to `depth` times, shifting the slots down after each
    rejected trial (the last slot keeps its value); the cap is tested after each trial."""
    trials = 0
    while True:
        slots, skip = [], False
        for r in range(depth):
            if skip:
                slots.append(EMPTY)  # zeroed slot: never decided, as a sure trial accepts
                continue
            t = trials + r
            slots.append(t)
            skip = sure[t]
        for _ in range(depth):
            t = slots[0]
            assert t is not EMPTY, "decided a zeroed slot"
            a = acc[t]
            trials += 1
            if a:
                return "acc", trials
            if trials >= cap:
                return "rvs", trials
            slots = slots[1:] + slots[-1:]


@pytest.mark.parametrize("depth", [1, 2, 3, 4, 5])
def test_batch_depths_equal_sequential(depth):
    rng = np.random.default_rng(100 + depth)
    cases = 0
    for cap in range(1, 14):
        for p_acc in (0.0, 0.05, 0.3, 0.7):
            for _ in range(200):
                n = cap + depth + 1
                acc = rng.random(n) < p_acc
                # a sure trial is an accepted one whose uniforms alone decide it
                sure = acc & (rng.random(n) < 0.5)
                assert batched(acc, sure, cap, depth) == sequential(acc, cap), (depth, cap, acc, sure)
                cases += 1
    assert cases == 13 * 4 * 200


def test_batch_fallback_on_batch_boundaries():
    """Caps that are multiples of the depth, one less and one more, with no acceptance."""
    for depth in range(1, 6):
        for cap in (depth - 1, depth, depth + 1, 2 * depth, 2 * depth + 1):
            if cap < 1:
                continue
            acc = np.zeros(cap + depth + 1, bool)
            assert batched(acc, acc, cap, depth) == ("rvs", cap)
            acc[cap - 1] = True  # accepted on the last trial the cap allows
            assert batched(acc, acc, cap, depth) == ("acc", cap)
            acc[cap - 1] = False
            acc[cap] = True  # one trial too late: the step falls back
            assert batched(acc, acc, cap, depth) == ("rvs", cap)
