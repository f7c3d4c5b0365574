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


def fake_run(monkeypatch, n, schedule, s, a, depth, pairs=True, triples=True):
    """A _Run whose launches are no-ops: only its host logic runs (which steps go into one-, two-
    and three-step launches, which reverse steps are paired, the byte count of each launch)."""
    import torch

    import paper_2002_05265_amd.adjoint as A

    for name in ("lbm_step_raw_many", "lbm_step2_raw_many", "lbm_step3_raw_many", "lbm_adjoint_many"):
        monkeypatch.setattr(A.B, name, lambda *args, **kw: None)
    r = A._Run.__new__(A._Run)
    r.ctx, r.model, r.omega = None, 3, [1.0] * 5
    r.s, r.a, r.reverse_depth = s, a, depth
    r.node_bytes = r.steps_run = r.nbuf = r.peak_states = 0
    r.schedule, r.nsteps = schedule, n
    r.saved, r.refs = {}, {}
    r.pool = [torch.empty(1, dtype=torch.uint8) for _ in range(n + 8)]
    r._two_step = lambda: pairs
    r._three_step = lambda: triples
    r.cur = r._free_buffer()
    r.lam = [torch.empty(1) for _ in range(3)]
    return r


@pytest.mark.parametrize("s,a", [(4, 4), (8, 8), (2, 4)])
def test_sweep_bytes(monkeypatch, s, a):
    # sqrt(n), n = 9: checkpoints every 3 steps.  Forward: three three-step launches, no state
    # between kept (3 x 18 s).  Backward, per segment: one two-step launch that also writes the
    # state between (27 s), then a pair of reverse steps (both states, lambda_{n+1} gathered,
    # lambda_{n-1} written: 18 s + 18 a) and one reverse step (9 s + 18 a).
    r = fake_run(monkeypatch, 9, "sqrt", s, a, 2)
    r._forward_fast()
    assert r.node_bytes == 3 * 18 * s
    r._backward_fast()
    assert r.steps_run == 9 + 6
    assert r.node_bytes == 3 * 18 * s + 3 * (27 * s + (18 * s + 18 * a) + (9 * s + 18 * a))
    # store-all, n = 9: every state kept, so four two-step launches writing the state between and
    # one single step; reverse: four pairs and one single, or nine singles with one per launch
    for depth, reverse in ((2, 4 * 18 * (s + a) + 9 * s + 18 * a), (1, 9 * (9 * s + 18 * a))):
        r = fake_run(monkeypatch, 9, "store_all", s, a, depth)
        r._forward_fast()
        assert r.node_bytes == 4 * 27 * s + 18 * s
        r._backward_fast()
        assert r.node_bytes == 4 * 27 * s + 18 * s + reverse
    # one step per launch: 18 s per step in both sweeps
    r = fake_run(monkeypatch, 9, "sqrt", s, a, 1, pairs=False, triples=False)
    r._forward_fast()
    r._backward_fast()
    assert r.node_bytes == (9 + 6) * 18 * s + 9 * (9 * s + 18 * a)
