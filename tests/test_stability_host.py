"""Host logic of the stability-map driver: the check schedule and the map reduction (no GPU)."""
import numpy as np

from paper_2002_05265_amd import inputs
from paper_2002_05265_amd import stability as S


def test_check_schedule_covers_every_budget():
    rng = np.random.default_rng(3)
    for _ in range(50):
        budgets = rng.integers(1, 5000, size=rng.integers(1, 20))
        every = int(rng.integers(1, 200))
        sched = S.check_schedule(budgets, every)
        assert sched[-1] == budgets.max()
        assert all(b in sched for b in budgets)
        gaps = np.diff([0] + sched)
        assert np.all(gaps > 0) and np.all(gaps <= every)
        # each check is a run's budget or comes exactly `every` steps after the previous one
        prev = 0
        for s in sched:
            assert s in budgets or s - prev == every
            prev = s


def test_vortex_budgets_are_m_convective_times():
    insts = S.vortex_instances(["BGK", "K"], ["SRT", "REG"], [1e-5, 1e-3], [0.1, 0.5], L=32, M=50)
    assert len(insts) == 16
    for d in insts:
        tc = 32 / (d["mach"] * inputs.CS)
        assert d["budget"] == int(np.ceil(50 * tc))
        assert np.allclose(d["omega"], inputs.rates(d["nu"], d["preset"]))


def test_max_stable_mach_stops_at_first_unstable():
    insts = S.vortex_instances(["BGK"], ["SRT"], [1e-4], [0.1, 0.2, 0.3, 0.4], L=32, M=1)
    # stable, stable, unstable, stable (an isolated stable point above the first failure)
    fb = np.array([-1, -1, 100, -1])
    assert S.max_stable_mach(insts, fb)[("BGK", "SRT", 1e-4)] == 0.2
    assert S.max_stable_mach(insts, np.array([5, -1, -1, -1]))[("BGK", "SRT", 1e-4)] == 0.0
