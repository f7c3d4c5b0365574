"""Host logic of the adjoint's checkpoint schedules (no GPU): replaying the actions on a fake
state machine must give one reverse step at each of the states n-1, ..., 0, in that order, each
at the right state, within the stated memory, and with the expected amount of recomputation."""
import math

import pytest

from paper_2002_05265_amd.adjoint import backward_actions, forward_actions, revolve_split


def replay(n, schedule, slots=0):
    cur, saved, steps, peak = 0, {}, 0, 0
    visited = []
    for act in list(forward_actions(n, schedule)):
        if act[0] == "save":
            saved[act[1]] = cur
        else:
            cur += act[1]
            steps += act[1]
        peak = max(peak, len(saved))
    assert cur == n
    for act in backward_actions(n, schedule, slots):
        kind = act[0]
        if kind == "save":
            saved[act[1]] = cur
            peak = max(peak, len(saved))
        elif kind == "advance":
            cur += act[1]
            steps += act[1]
        elif kind == "load":
            assert saved[act[1]] == act[2]
            cur = act[2]
        elif kind == "free":
            del saved[act[1]]
        else:
            visited.append(cur if act[1] is None else saved[act[1]])
    return visited, steps, peak


@pytest.mark.parametrize("n", [1, 2, 3, 7, 45, 100, 2000])
@pytest.mark.parametrize("schedule,slots", [("sqrt", 0), ("store_all", 0), ("revolve", 1), ("revolve", 3),
                                            ("revolve", 8)])
def test_reverse_order_and_memory(n, schedule, slots):
    if schedule == "revolve" and slots == 1 and n > 200:
        pytest.skip("one slot is quadratic")
    visited, steps, peak = replay(n, schedule, slots)
    assert visited == list(range(n - 1, -1, -1))
    if schedule == "sqrt":
        K = math.isqrt(max(n - 1, 0)) + 1 if n > 1 else 1
        assert peak <= math.ceil(n / K) + K
        assert steps <= 2 * n
    elif schedule == "store_all":
        assert peak == n and steps == n
    else:
        assert peak <= slots
        if slots >= 2:
            # binomial bound: one slot holds the initial state, so c = slots - 1 are free and
            # r repetitions suffice once C(c + r, c) >= n; every step then runs at most r + 1
            # times (the first forward sweep included)
            c, r = slots - 1, 0
            while math.comb(c + r, c) < n:
                r += 1
            assert steps <= (r + 1) * n


def test_revolve_split_respects_binomial_bound():
    for length in range(2, 300):
        for free in range(1, 6):
            m = revolve_split(length, free)
            assert 1 <= m < length
