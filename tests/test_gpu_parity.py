"""GPU parity: the HIP stream-and-collide path (through the C ABI) against the CPU oracle.

Bars: streaming bit-exact; FP64 within 1e-12 and shifted FP32 within 1e-5, normwise relative
(max-abs difference over max magnitude) on the populations f, the density rho and each
velocity component; FP16 storage within a bound derived from its unit roundoff (see
test_models_fp16).  The density deviation rho - rho0 is a tiny field (1e-4 of rho for a weak
vortex), so it is held to an absolute bound instead (see test_models_fp32_shifted).  Grids are
ragged with respect to the 64-lane wave and the 256-thread block so that tails are exercised.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.sim import Sim

pytestmark = pytest.mark.gpu

MODELS = list(inputs.MODEL_NAMES)
CENTRAL = {"CM", "CHM", "K"}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def orders(name):
    return [4] if name in CENTRAL else [2, 3, 4]


def omega_sets():
    rng = np.random.default_rng(99)
    return {"SRT": inputs.rates(1e-5, "SRT"), "REG": inputs.rates(1e-5, "REG"),
            "custom": np.array([1.97, *rng.uniform(0.3, 1.9, 4)])}


def test_stream_only_bit_exact(gpu):
    rng = np.random.default_rng(1)
    for nx, ny in [(64, 64), (97, 45), (3, 130)]:
        for prec in ("f64", "f32", "f16"):
            print(f"stream-only {nx}x{ny} {prec}", flush=True)
            rho, ux, uy = inputs.vortex_fields(nx, ny, 0.2)
            sim = Sim(rho, ux, uy, prec=prec, device=gpu)
            f = oracle.init_eq(4, rho, ux, uy) * (1 + 0.01 * rng.standard_normal((9, ny, nx)))
            sim.set_state(f, 0)
            s0 = sim.state().cpu().numpy()
            sim.step("STREAM_ONLY", [1.0] * 5, 7)
            s7 = sim.state().cpu().numpy()
            for i in range(9):
                np.testing.assert_array_equal(s7[i], np.roll(s0[i], (7 * oracle.CY[i], 7 * oracle.CX[i]), axis=(0, 1)))
            sim.step("STREAM_ONLY", [1.0] * 5, int(np.lcm(nx, ny)) - 7)
            np.testing.assert_array_equal(sim.state().cpu().numpy(), s0)
            if prec == "f64":
                np.testing.assert_array_equal(s0, f)
                np.testing.assert_array_equal(s7, oracle.step(f, oracle.STREAM_ONLY, 4, [1.0] * 5, 7))
            sim.close()


def test_c1_bgk_second_order_vortex(gpu):
    # 64 x 64, BGK with the second-order equilibrium, Ma = 0.1, beta = 0.15, R = 0.1 L,
    # nu = 1e-3, 200 steps: rho, u fields and total mass / kinetic energy
    n, steps = 64, 200
    rho, ux, uy = inputs.vortex_fields(n, n, 0.1, beta=0.15, radius_frac=0.1)
    omega = inputs.rates(1e-3, "SRT")
    sim = Sim(rho, ux, uy, prec="f64", eq_order=2, device=gpu)
    sim.step("BGK", omega, steps)
    r, u, v, tot = sim.moments()
    ref = oracle.step(oracle.init_eq(2, rho, ux, uy), oracle.BGK, 2, omega, steps)
    rr, ru, rv, rtot = oracle.moments(ref)
    assert rel(r.cpu().numpy(), rr) < 1e-12
    assert rel(u.cpu().numpy(), ru) < 1e-12
    assert rel(v.cpu().numpy(), rv) < 1e-12
    assert abs(tot[0] - rtot[0]) / rtot[0] < 1e-12
    assert abs(tot[3] - rtot[3]) / rtot[3] < 1e-12
    assert abs(tot[4] - rtot[4]) / rtot[4] < 1e-12
    assert tot[5] == steps
    assert rel(sim.state().cpu().numpy(), ref) < 1e-12
    assert sim.status() == (steps, -1)


@pytest.mark.parametrize("name", MODELS)
def test_models_fp64(gpu, name):
    nx, ny, steps = 70, 45, 40
    rho, ux, uy = inputs.vortex_fields(nx, ny, 0.3, beta=0.5, radius_frac=0.15)
    for N in orders(name):
        f0 = oracle.init_eq(N, rho, ux, uy)
        for preset, omega in omega_sets().items():
            print(f"{name} N={N} {preset}", flush=True)
            sim = Sim(rho, ux, uy, prec="f64", eq_order=N, device=gpu)
            sim.step(name, omega, steps)
            g = sim.state().cpu().numpy()
            r, u, v, tot = sim.moments()
            sim.close()
            ref = oracle.step(f0, inputs.MODEL_CODES[name], N, omega, steps)
            rr, ru, rv, rtot = oracle.moments(ref)
            assert rel(g, ref) < 1e-12, (name, N, preset, rel(g, ref))
            assert rel(r.cpu().numpy(), rr) < 1e-12
            assert rel(u.cpu().numpy(), ru) < 1e-12 and rel(v.cpu().numpy(), rv) < 1e-12
            assert abs(tot[0] - rtot[0]) < 1e-12 * rtot[0]


@pytest.mark.parametrize("name", MODELS)
@pytest.mark.parametrize("reference", ["rest", "mean-flow"])
def test_models_fp32_shifted(gpu, name, reference):
    nx, ny, steps = 70, 45, 40
    rho, ux, uy = inputs.vortex_fields(nx, ny, 0.3, beta=0.5, radius_frac=0.15)
    omega = omega_sets()["REG"]
    ref = oracle.step(oracle.init_eq(4, rho, ux, uy), inputs.MODEL_CODES[name], 4, omega, steps)
    rr, ru, rv, _ = oracle.moments(ref)
    uref = (0.0, 0.0) if reference == "rest" else (0.3 * inputs.CS, 0.0)
    sim = Sim(rho, ux, uy, prec="f32", eq_order=4, device=gpu, ref_velocity=uref)
    sim.step(name, omega, steps)
    r, u, v, _ = sim.moments()
    g = sim.state().cpu().numpy()
    r = r.cpu().numpy()
    e = [rel(g, ref), rel(r, rr), rel(u.cpu().numpy(), ru), rel(v.cpu().numpy(), rv)]
    drho = float(np.max(np.abs(r - rr)))
    print(name, reference, "fp32 errors f, rho, ux, uy", e, "max |d rho|", drho, flush=True)
    assert max(e) < 1e-5, e
    # each stored deviation carries a rounding of at most 2^-24 |h| (|h| <= 0.09 here); mass
    # errors are never damped, and the nine roundings per node and step random-walk over the
    # run: |d rho| <~ 4 sigma ~ 4 * sqrt(9 * steps) * 2^-24 * 0.09 ~ 4.1e-7 (max over nodes)
    assert drho < 5e-7, drho


@pytest.mark.parametrize("name", [m for m in MODELS if m not in CENTRAL])
@pytest.mark.parametrize("N", [2, 3])
def test_models_fp32_shifted_lower_orders(gpu, name, N):
    # the truncated equilibria of reading 3 in the shifted storage, whose reference state is then
    # the truncated f^eq_N(rho0, U) too: mean-flow reference, the same bars as at N = 4
    nx, ny, steps = 70, 45, 40
    rho, ux, uy = inputs.vortex_fields(nx, ny, 0.3, beta=0.5, radius_frac=0.15)
    omega = omega_sets()["custom"]
    ref = oracle.step(oracle.init_eq(N, rho, ux, uy), inputs.MODEL_CODES[name], N, omega, steps)
    _, ru, rv, _ = oracle.moments(ref)
    sim = Sim(rho, ux, uy, prec="f32", eq_order=N, device=gpu, ref_velocity=(0.3 * inputs.CS, 0.0))
    sim.step(name, omega, steps)
    _, u, v, _ = sim.moments()
    g = sim.state().cpu().numpy()
    sim.close()
    e = [rel(g, ref), rel(u.cpu().numpy(), ru), rel(v.cpu().numpy(), rv)]
    print(name, N, "fp32 errors f, ux, uy", e, flush=True)
    assert max(e) < 1e-5, e


@pytest.mark.parametrize("name", ["BGK", "CM", "K", "RR"])
@pytest.mark.parametrize("reference", ["rest", "mean-flow"])
def test_models_fp16(gpu, name, reference):
    # FP16 storage rounds every stored deviation h_i with relative error <= 2^-11; over 40
    # steps the accumulated error stays within 40 * 2^-11 * max|h| / max|u| ~ 2e-2 of the
    # velocity scale, the bound asserted here.
    nx, ny, steps = 70, 45, 40
    rho, ux, uy = inputs.vortex_fields(nx, ny, 0.3, beta=0.5, radius_frac=0.15)
    omega = omega_sets()["REG"]
    ref = oracle.step(oracle.init_eq(4, rho, ux, uy), inputs.MODEL_CODES[name], 4, omega, steps)
    _, ru, rv, _ = oracle.moments(ref)
    uref = (0.0, 0.0) if reference == "rest" else (0.3 * inputs.CS, 0.0)
    sim = Sim(rho, ux, uy, prec="f16", eq_order=4, device=gpu, ref_velocity=uref)
    sim.step(name, omega, steps)
    _, u, v, _ = sim.moments()
    e = [rel(u.cpu().numpy(), ru), rel(v.cpu().numpy(), rv)]
    print(name, reference, "fp16 errors", e, flush=True)
    assert max(e) < 2e-2, e


def test_state_roundtrip_and_resume(gpu):
    rho, ux, uy = inputs.vortex_fields(66, 50, 0.25)
    omega = inputs.rates(1e-4, "REG")
    for prec in ("f64", "f32"):
        sim = Sim(rho, ux, uy, prec=prec, device=gpu)
        sim.step("K", omega, 10)
        saved = sim.state()
        sim.step("K", omega, 15)
        a = sim.state().cpu().numpy()
        sim.set_state(saved, 10)
        assert sim.status()[0] == 10
        sim.step("K", omega, 15)
        b = sim.state().cpu().numpy()
        np.testing.assert_array_equal(a, b)
        sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_degenerate_grids_and_rates(gpu, prec):
    # the smallest grids (every neighbour wraps onto the node itself or its single partner), very
    # thin ones, rates at the ends of [0, 2], and zero-step calls
    rng = np.random.default_rng(5)
    bar = 1e-12 if prec == "f64" else 1e-5
    for nx, ny in [(2, 2), (2, 17), (19, 2), (3, 3), (257, 2)]:
        rho = 1.0 + 0.01 * rng.standard_normal((ny, nx))
        ux = 0.05 * rng.standard_normal((ny, nx))
        uy = 0.05 * rng.standard_normal((ny, nx))
        for name in MODELS:
            N = 4
            f0 = oracle.init_eq(N, rho, ux, uy)
            for omega in ([0.0] * 5, [2.0] * 5, [1.0, 0.0, 2.0, 0.5, 1.5]):
                sim = Sim(rho, ux, uy, prec=prec, eq_order=N, device=gpu)
                sim.step(name, omega, 0)
                np.testing.assert_allclose(sim.state().cpu().numpy(), f0, rtol=0, atol=1e-15 if prec == "f64" else 1e-7)
                sim.step(name, omega, 7)
                g = sim.state().cpu().numpy()
                sim.close()
                ref = oracle.step(f0, inputs.MODEL_CODES[name], N, omega, 7)
                e = rel(g, ref)
                assert e < bar, (nx, ny, name, omega, prec, e)


def test_blowup_flag(gpu):
    n = 40
    rho, ux, uy = inputs.vortex_fields(n, n, 0.1)
    omega = inputs.rates(1e-3, "SRT")
    sim = Sim(rho, ux, uy, prec="f64", device=gpu)
    sim.step("BGK", omega, 5)
    assert sim.status() == (5, -1)
    f = oracle.init_eq(4, rho, ux, uy)
    f[3, 7, 11] = np.nan
    sim.set_state(f, 20)
    assert sim.status() == (20, -1)
    sim.step("BGK", omega, 3)
    assert sim.status() == (23, 20)
    g = oracle.init_eq(4, rho, ux, uy)
    g[:, 2, 2] = -0.1  # a node with rho < 0
    for prec in ("f64", "f32", "f16"):
        s2 = Sim(rho, ux, uy, prec=prec, device=gpu)
        s2.set_state(g, 0)
        s2.step("RR", omega, 2)
        assert s2.status() == (2, 0), prec
        s2.close()


def test_srt_and_reg_identities_on_gpu(gpu):
    n, steps = 256, 100
    rho, ux, uy = inputs.vortex_fields(n, n, 0.3, beta=0.5)
    srt, reg = inputs.rates(1e-5, "SRT"), inputs.rates(1e-5, "REG")

    def run(name, omega):
        s = Sim(rho, ux, uy, prec="f64", device=gpu)
        s.step(name, omega, steps)
        out = s.state().cpu().numpy()
        s.close()
        return out

    bgk = run("BGK", srt)
    for name in ("RM", "HM", "CM", "CHM"):
        assert rel(run(name, srt), bgk) < 1e-12, name
    assert rel(run("K", srt), bgk) > 1e-10
    pr = run("PR", reg)
    assert rel(run("HM", reg), pr) < 1e-12 and rel(run("RR", reg), pr) < 1e-12
    assert rel(run("CHM", reg), run("RR", srt)) < 1e-12


def test_argument_errors_on_gpu(gpu):
    rho, ux, uy = inputs.vortex_fields(16, 16, 0.1)
    s = Sim(rho, ux, uy, prec="f64", eq_order=2, device=gpu)
    import paper_2002_05265_amd.binding as B

    with pytest.raises(B.LbmError) as e:
        s.step("CM", [1.9] * 5, 1)
    assert e.value.code == -2
    with pytest.raises(B.LbmError) as e:
        s.step("BGK", [2.5, 1, 1, 1, 1], 1)
    assert e.value.code == -1
    with pytest.raises(B.LbmError):
        s.step(42, [1.0] * 5, 1)
    assert s.status() == (0, -1)
    s.close()


def test_argument_errors_of_two_step_and_dvbe_entry_points(gpu):
    import torch

    import paper_2002_05265_amd.binding as B
    from paper_2002_05265_amd import lsa

    rho, ux, uy = inputs.vortex_fields(16, 16, 0.1)
    s = Sim(rho, ux, uy, prec="f64", device=gpu)
    n = B.lbm_state_bytes(s.ctx)
    a, b, c = (torch.empty(n, dtype=torch.uint8, device=gpu) for _ in range(3))
    w = [1.5] * 5
    # a pair's three buffers must differ; counts and steps in range
    for src, mid, dst in ((a, None, a), (a, a, b), (a, b, b)):
        with pytest.raises(B.LbmError) as e:
            B.lbm_step2_raw_many(s.ctx, 0, w, [src.data_ptr()], None if mid is None else [mid.data_ptr()],
                                 [dst.data_ptr()], 0)
        assert e.value.code == -1
    with pytest.raises(B.LbmError):
        B.lbm_step2_raw_many(s.ctx, 0, w, [a.data_ptr()], None, [b.data_ptr()], -1)
    with pytest.raises(B.LbmError):
        B.lbm_step2_raw_many(s.ctx, 42, w, [a.data_ptr()], None, [b.data_ptr()], 0)  # unknown model
    B.lbm_save_state(s.ctx, a.data_ptr())
    B.lbm_step2_raw_many(s.ctx, 0, w, [], None, [], 0)  # an empty call does nothing
    B.lbm_step2_raw_many(s.ctx, 0, w, [a.data_ptr()], [c.data_ptr()], [b.data_ptr()], 0)
    s.close()
    # DVBE: tau must be positive; the points are checked
    kx = torch.zeros(4, dtype=torch.float64, device=gpu)
    pt = lsa.point("BGK", 0.0, 0.1, eq_order=2, omega=[1.0] * 5)
    for tau in (0.0, -1.0, float("nan")):
        with pytest.raises(B.LbmError):
            lsa.dvbe_growth([pt], kx, kx, tau=tau)
    bad = dict(pt, eq_order=5)
    with pytest.raises(B.LbmError):
        lsa.dvbe_growth([bad], kx, kx)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_third_order_equilibrium_default_launch(gpu, prec):
    # N = 3 (A21, A12 kept, A22 = 0) on a grid large enough for the default launch of three steps
    # per launch, 7 steps (two three-step launches and a single step)
    nx, ny, steps = 520, 512, 7
    rho, ux, uy = inputs.vortex_fields(nx, ny, 0.3, beta=0.5, radius_frac=0.15)
    f0 = oracle.init_eq(3, rho, ux, uy)
    for name in ("BGK", "RM", "HM", "PR", "RR"):
        omega = omega_sets()["custom"]
        print(f"{name} N=3 {prec} {nx}x{ny}", flush=True)
        sim = Sim(rho, ux, uy, prec=prec, eq_order=3, device=gpu)
        assert sim.fusion_depth(name) == 3
        sim.step(name, omega, steps)
        g = sim.state().cpu().numpy()
        sim.close()
        ref = oracle.step(f0, inputs.MODEL_CODES[name], 3, omega, steps)
        assert rel(g, ref) < (1e-12 if prec == "f64" else 1e-5), (name, rel(g, ref))
