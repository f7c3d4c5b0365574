"""Studies of Section 5d and Appendix C, run on the batched kernel.

Double shear layer (Appendix C; Ma = u0 / cs, Re = u0 L / nu = 3e4, the analytic roll-up initial
condition; the paper's own initialisation is not given, so the comparison is qualitative):
- PR at Ma = 0.12 becomes unstable sooner the finer the grid (the paper: stable to 2 t_c at
  L = 128, unstable near 1.8 t_c at L = 256 and 1.7 t_c at L = 512);
- the largest stable Ma over 3 t_c does not grow with the resolution, and RR is stable to several
  times the Mach number of PR (the paper quotes 0.14 / 0.11 for PR and 0.52 / 0.49 for RR at
  L = 128 / 256).
Long-distance transport (Section 5d; convected vortex, Ma = 0.5, nu = 1e-4, 50 convective times):
- REG-CHM gives the vorticity field of SRT-RR (the two operators coincide);
- REG-K is as accurate as SRT-RR; doubling the resolution reduces the error and the dissipation.
"""
import numpy as np
import pytest

from paper_2002_05265_amd import accuracy as A
from paper_2002_05265_amd import inputs
from paper_2002_05265_amd import stability as S

pytestmark = pytest.mark.gpu


def test_dsl_pr_finer_grid_is_unstable_sooner(gpu):
    inst = S.dsl_instances([("PR", "REG")], [128, 256, 512], [0.12], M=3)
    fb, _, _ = S.run_stability(inst, field=S.dsl_field, device=gpu)
    tc = np.array([d["nx"] / (0.12 * inputs.CS) for d in inst])
    t = np.where(fb >= 0, fb / tc, np.inf)
    print("PR Ma 0.12: instability at t / t_c =", dict(zip((128, 256, 512), t.round(3))), flush=True)
    assert t[1] < 3 and t[2] < 3          # 256 and 512 become unstable within 3 t_c
    assert t[0] > t[1] > t[2]              # sooner on finer grids (128 may stay stable)
    assert 1.0 < t[2] and 1.0 < t[1]       # after the roll-up has started, not at the start


def test_dsl_max_stable_mach(gpu):
    machs = [round(0.02 * k, 2) for k in range(2, 36)]
    inst = S.dsl_instances([("PR", "REG"), ("RR", "SRT")], [128, 256], machs, M=3)
    fb, _, _ = S.run_stability(inst, field=S.dsl_field, device=gpu)
    best = {}
    for d, f in zip(inst, fb):
        best.setdefault((d["model"], d["nx"]), []).append((d["mach"], f))
    ms = {}
    for key, pts in best.items():
        ms[key] = 0.0
        for ma, f in sorted(pts):
            if f >= 0:
                break
            ms[key] = ma
    print("largest stable Ma over 3 t_c:", ms, flush=True)
    for m in ("PR", "RR"):
        assert ms[(m, 256)] <= ms[(m, 128)]
    for L in (128, 256):
        assert ms[("RR", L)] >= 3 * ms[("PR", L)] > 0


def test_long_distance_transport(gpu):
    res, _ = A.transport_accuracy([("RR", "SRT"), ("CHM", "REG"), ("K", "REG")], [256, 512], device=gpu)
    for key, v in res.items():
        print(key, {k: v[k] for k in ("l2", "peak", "shift", "blowup")}, flush=True)
        assert v["blowup"] < 0
    for L in (256, 512):
        a, b = res[("RR", "SRT", L)]["w"], res[("CHM", "REG", L)]["w"]
        d = float((a - b).abs().max() / a.abs().max())
        print(f"L={L}: REG-CHM vs SRT-RR vorticity {d:.2e}", flush=True)
        # the same map up to rounding: ~1e-16 per step over 44k / 89k steps of a stable flow
        assert d < 1e-9
        rr, k = res[("RR", "SRT", L)], res[("K", "REG", L)]
        assert abs(k["l2"] - rr["l2"]) < 0.01 * rr["l2"]
    for m, p in (("RR", "SRT"), ("K", "REG")):
        lo, hi = res[(m, p, 256)], res[(m, p, 512)]
        assert hi["l2"] < lo["l2"] and abs(1 - hi["peak"]) < abs(1 - lo["peak"])
        assert np.hypot(*hi["shift"]) < np.hypot(*lo["shift"])
