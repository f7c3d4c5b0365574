"""Two steps per launch (lbm_set_fusion, temporal blocking through an LDS ring) against single
steps: the same arithmetic per node and the stored type in the ring, so states, step counters and
blow-up steps are bit-identical, for every model, precision, ring and strip height, on grids
ragged against the 64-column strip and the strip height, on grids narrower than a strip or
shorter than the ring, and for odd step counts (the last step single).  One case is also checked
against the oracle directly.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.sim import Sim

pytestmark = pytest.mark.gpu

MODELS = list(inputs.MODEL_NAMES) + ["STREAM_ONLY"]


def perturbed(nx, ny, seed):
    rng = np.random.default_rng(seed)
    rho, ux, uy = inputs.vortex_fields(nx, ny, 0.3)
    return (rho * (1 + 0.02 * rng.standard_normal((ny, nx))), ux + 0.02 * rng.standard_normal((ny, nx)),
            uy + 0.02 * rng.standard_normal((ny, nx)))


def run_pair(gpu, prec, model, nx, ny, ring, strip, nsteps, omega, seed=5):
    rho, ux, uy = perturbed(nx, ny, seed)
    a = Sim(rho, ux, uy, prec=prec, device=gpu)
    b = Sim(rho, ux, uy, prec=prec, device=gpu)
    a.set_fusion(model, 0)  # single steps
    b.set_fusion(model, ring, strip)
    b.set_fusion_depth(model, 2)  # the two-step kernel (a new context may default to three)
    a.step(model, omega, nsteps)
    b.step(model, omega, nsteps)
    sa, sb = a.state().cpu().numpy(), b.state().cpu().numpy()
    st = (a.status(), b.status())
    a.close()
    b.close()
    return sa, sb, st


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_bit_identical_to_single_steps(gpu, prec):
    rng = np.random.default_rng(11)
    cases = [(200, 70, 8, 32), (130, 37, 16, 16), (64, 8, 4, 8), (70, 3, 8, 64), (5, 21, 16, 32), (2, 2, 4, 4),
             (131, 66, 4, 12)]
    for k, model in enumerate(MODELS):
        omega = inputs.rates(1e-4, "REG") if k % 2 else np.array([1.9, *rng.uniform(0.4, 1.9, 4)])
        nx, ny, ring, strip = cases[k % len(cases)]
        for nsteps in (6, 7):
            print(f"{prec} {model} {nx}x{ny} ring {ring} strip {strip} steps {nsteps}", flush=True)
            sa, sb, (ta, tb) = run_pair(gpu, prec, model, nx, ny, ring, strip, nsteps, omega)
            np.testing.assert_array_equal(sa, sb)
            assert ta == tb


def test_every_shape_on_one_model(gpu):
    omega = inputs.rates(1e-5, "REG")
    for nx, ny in ((257, 131), (64, 64), (63, 17)):
        for ring in (4, 8, 16):
            for strip in (ring, 2 * ring, 8 * ring, 1024):
                strip -= strip % ring
                print(f"CM f32 {nx}x{ny} ring {ring} strip {strip}", flush=True)
                sa, sb, (ta, tb) = run_pair(gpu, "f32", "CM", nx, ny, ring, strip, 4, omega)
                np.testing.assert_array_equal(sa, sb)
                assert ta == tb


def test_blowup_step_matches(gpu):
    # a node with f_1 = 5, f_3 = -4 (rho > 0 there) and zero rates: one step later its left
    # neighbour holds f_3 = -4 and rho < 0, so the first bad state is n + 1 (the second step of a
    # pair); placed on strip and grid edges so that halo nodes see it first
    nx, ny = 130, 40
    f = oracle.init_eq(4, np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    for ax, ay in ((64, 16), (0, 0), (63, 39), (129, 7)):
        g = f.copy()
        g[1, ay, ax], g[3, ay, ax] = 5.0, -4.0
        for prec in ("f64", "f32"):
            for model in ("BGK", "STREAM_ONLY"):
                out = []
                for fused in (False, True):
                    s = Sim(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), prec=prec, device=gpu)
                    if fused:
                        s.set_fusion(model, 8, 16)
                    s.set_state(g, 10)
                    s.step(model, [0.0] * 5, 3)
                    out.append(s.status())
                    s.close()
                assert out[0] == out[1] == (13, 11), (ax, ay, prec, model, out)


def test_against_oracle(gpu):
    nx, ny = 70, 40
    rho, ux, uy = perturbed(nx, ny, 3)
    omega = np.array([1.7, 1.2, 0.9, 1.4, 1.1])
    s = Sim(rho, ux, uy, prec="f64", device=gpu)
    s.set_fusion("K", 8, 16)
    s.step("K", omega, 5)
    got = s.state().cpu().numpy()
    s.close()
    ref = oracle.step(oracle.init_eq(4, rho, ux, uy), inputs.MODEL_CODES["K"], 4, omega, 5)
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert err < 1e-12, err


def test_rejects_bad_shapes(gpu):
    rho, ux, uy = perturbed(16, 16, 1)
    s = Sim(rho, ux, uy, prec="f32", device=gpu)
    for ring, strip in ((6, 12), (8, 12), (16, 8), (8, 0), (32, 64)):
        with pytest.raises(RuntimeError):
            s.set_fusion("BGK", ring, strip)
    s.set_fusion("BGK", 0)
    s.close()


def deep_strip(nx, ny, prec):
    """Base strip height of a new context's three-step launches (include/lbm.h)."""
    gsx = (nx + 63) // 64
    h = 8 * int(gsx * ny / (nx * ny) ** 0.5 / 8.0 + 0.5)
    hs = min(max(h, 8), 64)
    return 128 if (prec == "f32" and hs == 64) else hs


def deep_pick(model, nx, ny, prec, cus):
    """(ring_rows, strip_rows) of a model's default three-step launches (include/lbm.h)."""
    hs = deep_strip(nx, ny, prec)
    if prec == "f64":
        return (8, 128 if hs == 64 else hs)
    gsx = (nx + 63) // 64
    rnd = 3 * cus

    def strips(r):
        return gsx * (-(-ny // r))

    h = hs
    if strips(h) > rnd and 2 * strips(h) <= 3 * rnd:
        while strips(h) > rnd and h < 256:
            h += 8
    return (8, h)


def test_defaults_and_autotune(gpu):
    # a new context's fused setting follows the strip counts (include/lbm.h): three steps per
    # launch (FP32, FP64) from 512 strips of 64 columns on, else the two-step rule
    for (nx, ny, prec), want in {(2048, 2048, "f32"): (8, 16), (2048, 2048, "f64"): (8, 64),
                                 (4096, 1024, "f16"): (8, 40), (512, 512, "f32"): (8, 16),
                                 (256, 256, "f32"): (0, 0), (2048, 1000, "f64"): (8, 16),
                                 (512, 512, "f16"): (0, 0), (448, 512, "f64"): (0, 0),
                                 (2048, 1024, "f32"): (8, 16), (1024, 2048, "f32"): (8, 16), (1024, 1024, "f32"): (8, 16),
                                 (4096, 4096, "f32"): (8, 16), (4096, 4096, "f64"): (8, 64),
                                 (4096, 4096, "f16"): (8, 40), (320, 256, "f32"): (0, 0),
                                 (3072, 1536, "f32"): (8, 16)}.items():
        rho, ux, uy = np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx))
        s = Sim(rho, ux, uy, prec=prec, device=gpu)
        got = [(s.fusion_depth(m), s.fusion(m)) for m in MODELS]
        s.close()
        hs = deep_strip(nx, ny, prec)
        deep = prec != "f16" and (nx + 63) // 64 * (-(-ny // hs)) >= 512
        exp = []
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        for m in MODELS:
            if deep:
                exp.append((3, deep_pick(m, nx, ny, prec, cus)))
                continue
            # two steps: FP32 models take their 128-column setting where it gives >= 1024 strips
            wr, ws = (8, 8) if m == "BGK" else (4, 20)
            wide = prec == "f32" and want[0] and (nx + 127) // 128 * (-(-ny // ws)) >= 1024
            exp.append((2, (wr, ws) if wide else want))
        assert got == exp, (nx, ny, prec, got)
        if (nx, ny, prec) == (4096, 4096, "f32"):
            assert exp[0] == (3, (8, 128))
        if (nx, ny, prec) == (4096, 4096, "f64"):
            assert exp[0] == (3, (8, 128)) and exp[5] == (3, (8, 128))
        if (nx, ny, prec) in ((256, 256, "f32"), (448, 512, "f64")):
            assert not deep
    # autotune leaves state and counter alone, keeps a valid choice, and results do not change
    nx, ny = 1024, 512
    rho, ux, uy = perturbed(nx, ny, 8)
    omega = inputs.rates(1e-5, "REG")
    a = Sim(rho, ux, uy, prec="f32", device=gpu)
    b = Sim(rho, ux, uy, prec="f32", device=gpu)
    a.step("RR", omega, 3)
    b.step("RR", omega, 3)
    before = a.state().cpu().numpy()
    rows, xcd, us = a.autotune("RR", omega, 2)
    ring, strip = a.fusion("RR")
    print(f"autotune 1024x512 RR: rows {rows} xcd {xcd} ring {ring} strip {strip} {us:.1f} us/step", flush=True)
    assert rows in (1, 2, 4) and xcd in (0, 1) and us > 0
    depth = a.fusion_depth("RR")
    if depth == 2:
        assert (ring, strip) in ((0, 0), (8, 8), (8, 16), (8, 40), (8, 64), (16, 16), (4, 16), (4, 20), (4, 64))
    else:
        assert depth == 3 and (ring, strip) in ((4, 8), (4, 16), (4, 32), (4, 64), (8, 8), (8, 16), (8, 24),
                                                (8, 32), (8, 64), (8, 80), (8, 96), (8, 128))
    np.testing.assert_array_equal(a.state().cpu().numpy(), before)
    assert a.status() == (3, -1)
    a.step("RR", omega, 9)
    b.step("RR", omega, 9)
    np.testing.assert_array_equal(a.state().cpu().numpy(), b.state().cpu().numpy())
    a.close()
    b.close()


def test_single_step_shapes_agree(gpu):
    nx, ny = 300, 77
    rho, ux, uy = perturbed(nx, ny, 9)
    omega = np.array([1.8, 1.3, 1.1, 0.9, 1.5])
    ref = None
    for rows in (1, 2, 4):
        for xcd in (0, 1):
            s = Sim(rho, ux, uy, prec="f32", device=gpu)
            s.set_fusion("CHM", 0)
            s.set_launch("CHM", rows, xcd)
            s.step("CHM", omega, 5)
            st = s.state().cpu().numpy()
            s.close()
            if ref is None:
                ref = st
            np.testing.assert_array_equal(st, ref)


def test_wide_strips_bit_identical(gpu):
    """FP32 models take 128-column strips once these give >= 1024 strips: a grid ragged
    against 128 columns and the strip height, every ring, plain and raw (with the state between)
    two-step launches against single steps."""
    import torch

    from paper_2002_05265_amd import binding as B

    nx, ny = 1030, 1100  # 9 x 138 strips of 128 x 8
    omega = np.array([1.93, 1.2, 1.05, 0.9, 1.4])
    for model in ("BGK", "K", "RR", "STREAM_ONLY"):
        for ring, strip, h in ((4, 4, ny), (4, 8, ny), (8, 8, ny), (16, 16, 2 * ny)):
            assert (nx + 127) // 128 * (-(-h // strip)) >= 1024
            print(f"wide strips f32 {model} ring {ring} strip {strip} {nx}x{h}", flush=True)
            sa, sb, (ta, tb) = run_pair(gpu, "f32", model, nx, h, ring, strip, 5, omega, seed=13)
            np.testing.assert_array_equal(sa, sb)
            assert ta == tb
    rho, ux, uy = perturbed(nx, ny, 14)
    s = Sim(rho, ux, uy, prec="f32", device=gpu)
    n = B.lbm_state_bytes(s.ctx)
    # zeroed: the plane padding is never written and must compare equal
    a, m1, b, c, d = (torch.zeros(n, dtype=torch.uint8, device=gpu) for _ in range(5))
    B.lbm_save_state(s.ctx, a.data_ptr())
    code = inputs.MODEL_CODES["PR"]
    B.lbm_set_fusion(s.ctx, code, 4, 8)
    B.lbm_step_raw_many(s.ctx, code, omega, [a.data_ptr(), c.data_ptr()], [c.data_ptr(), d.data_ptr()], 0)
    B.lbm_step2_raw_many(s.ctx, code, omega, [a.data_ptr()], [m1.data_ptr()], [b.data_ptr()], 0)
    torch.cuda.synchronize()
    assert torch.equal(m1, c) and torch.equal(b, d)
    s.close()
