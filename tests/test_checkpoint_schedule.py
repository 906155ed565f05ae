"""Binomial checkpoint schedules (host logic of fd_gradient, no GPU): every
schedule is executable and reverses the steps in order, each step is
computed for the first time exactly once, and the number of forward steps
equals the optimum -- the closed form of the binomial checkpointing theorem
(Griewank and Walther) and an exhaustive search on small cases.  The split
of each segment is the smallest optimal one of the exhaustive recurrence,
and schedules far longer than a table over all (length, slots) pairs could
hold are planned too."""
import functools
from math import comb

import pytest

from paper_1906_10811_amd import _lib

ADV, STO, RES, YOU = _lib.FD_ACT_ADVANCE, _lib.FD_ACT_STORE, _lib.FD_ACT_RESTORE, _lib.FD_ACT_YOUTURN


def simulate(nt, slots, acts):
    """Run the schedule on a state machine; return forward steps and the
    levels computed for the first time."""
    stored = {0: 0}           # slot -> level
    cur = 0
    fwd = 0
    turns = []
    first = []
    horizon = 0
    for kind, step, count, slot, is_first in acts:
        if kind == STO:
            assert cur == step and 1 <= slot <= slots
            stored[slot] = step
        elif kind == RES:
            assert stored.get(slot) == step, (slot, step, stored)
            cur = step
        elif kind == ADV:
            assert cur == step and count >= 1
            new = [n for n in range(step, step + count) if n >= horizon]
            assert bool(new) == bool(is_first)
            first += new
            horizon = max(horizon, step + count)
            cur = step + count
            fwd += count
        elif kind == YOU:
            assert cur == step and count == 1
            if step >= horizon:
                first.append(step)
                horizon = step + 1
                assert is_first
            turns.append(step)
        else:
            raise AssertionError(kind)
    assert turns == list(range(nt - 1, -1, -1))
    assert sorted(first) == list(range(nt))
    return fwd


def closed_form(l, slots):
    """Minimal forward steps to reverse l steps with c = slots + 1 checkpoints
    (the initial state included): r l - beta(c + 1, r - 1), r the least
    integer with beta(c, r) = C(c + r, c) >= l."""
    c = slots + 1
    r = 0
    while comb(c + r, c) < l:
        r += 1
    return r * l - comb(c + 1 + r - 1, c + 1)


@functools.lru_cache(maxsize=None)
def brute(l, c):
    """Exhaustive minimum over all split points (independent of the library)."""
    if l == 1:
        return 0
    if c == 0:
        return l * (l - 1) // 2
    return min(m + brute(l - m, c - 1) + brute(m, c) for m in range(1, l))


@pytest.mark.parametrize("nt,slots", [(1, 0), (1, 3), (2, 1), (7, 0), (10, 2), (37, 3), (100, 5), (250, 8),
                                      (800, 16)])
def test_schedule_valid_and_optimal(nt, slots):
    acts, fwd = _lib.checkpoint_schedule(nt, slots)
    assert simulate(nt, slots, acts) == fwd
    assert fwd == closed_form(nt, min(slots, nt))


def test_schedule_matches_exhaustive_search():
    for l in range(1, 16):
        for c in range(0, 5):
            _, fwd = _lib.checkpoint_schedule(l, c)
            assert fwd == brute(l, min(c, l)), (l, c)


def test_more_slots_never_cost_more():
    prev = None
    for slots in range(0, 12):
        _, fwd = _lib.checkpoint_schedule(300, slots)
        if prev is not None:
            assert fwd <= prev
        prev = fwd
    assert prev < 3 * 300


def test_first_split_is_the_smallest_optimal_one():
    """The first snapshot of a schedule is taken after the smallest m that
    minimises m + T(l - m, c - 1) + T(m, c) (exhaustive recurrence)."""
    for l in range(2, 40):
        for c in range(1, 6):
            acts, _ = _lib.checkpoint_schedule(l, c)
            cc = min(c, l)
            costs = [m + brute(l - m, cc - 1) + brute(m, cc) for m in range(1, l)]
            want = 1 + costs.index(min(costs))
            assert acts[0][0] == RES and acts[1][0] == ADV and acts[2][0] == STO, (l, c)
            assert acts[1][2] == want and acts[2][1] == want, (l, c, acts[1], want)


@pytest.mark.parametrize("nt,slots", [(20000, 30), (100000, 50)])
def test_long_schedules(nt, slots):
    acts, fwd = _lib.checkpoint_schedule(nt, slots)
    assert fwd == closed_form(nt, slots)
    assert simulate(nt, slots, acts) == fwd
