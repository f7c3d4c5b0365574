"""Three steps per launch (lbm_set_fusion_depth 3: two LDS rings) against single steps: the same
arithmetic per node and the stored type in both rings, so states, step counters and blow-up steps
are bit-identical, for every model, FP32 and FP64, both rings, grids ragged against the strip width and height,
narrower than a strip or lower than the ring (down to 2 x 2), and step counts that end in a pair
or a single step.  One case is also checked against the oracle."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.binding import LbmError
from paper_2002_05265_amd.sim import Sim

pytestmark = pytest.mark.gpu

MODELS = list(inputs.MODEL_NAMES) + ["STREAM_ONLY"]


def perturbed(nx, ny, seed):
    rng = np.random.default_rng(seed)
    rho, ux, uy = inputs.vortex_fields(nx, ny, 0.3)
    return (rho * (1 + 0.02 * rng.standard_normal((ny, nx))), ux + 0.02 * rng.standard_normal((ny, nx)),
            uy + 0.02 * rng.standard_normal((ny, nx)))


def run_triple(gpu, model, nx, ny, ring, strip, nsteps, omega, seed=7, fields=None, prec="f32"):
    rho, ux, uy = fields if fields is not None else perturbed(nx, ny, seed)
    a = Sim(rho, ux, uy, prec=prec, device=gpu)
    b = Sim(rho, ux, uy, prec=prec, device=gpu)
    a.set_fusion(model, 0)
    b.set_fusion(model, ring, strip)
    b.set_fusion_depth(model, 3)
    a.step(model, omega, nsteps)
    b.step(model, omega, nsteps)
    sa, sb = a.state().cpu().numpy(), b.state().cpu().numpy()
    st = (a.status(), b.status())
    a.close()
    b.close()
    return sa, sb, st


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_three_steps_bit_identical(gpu, prec):
    rng = np.random.default_rng(21)
    cases = [(200, 70, 8, 32), (130, 37, 4, 12), (64, 8, 4, 8), (70, 3, 8, 64), (5, 21, 4, 4), (2, 2, 4, 4),
             (131, 66, 8, 8), (3, 40, 8, 16), (257, 19, 4, 20)]
    for k, model in enumerate(MODELS):
        omega = inputs.rates(1e-4, "REG") if k % 2 else np.array([1.9, *rng.uniform(0.4, 1.9, 4)])
        for j in range(2):
            nx, ny, ring, strip = cases[(k + 4 * j) % len(cases)]
            for nsteps in (6, 7, 8):
                print(f"three steps {prec} {model} {nx}x{ny} ring {ring} strip {strip} steps {nsteps}", flush=True)
                sa, sb, (ta, tb) = run_triple(gpu, model, nx, ny, ring, strip, nsteps, omega, prec=prec)
                np.testing.assert_array_equal(sa, sb)
                assert ta == tb


def test_three_steps_large_grid(gpu):
    # many strips, ragged against 64 columns and the strip height, both rings
    nx = 1030
    omega = np.array([1.93, 1.2, 1.05, 0.9, 1.4])
    for model, ring, strip, ny, prec in (("BGK", 8, 40, 1100, "f32"), ("K", 4, 12, 1100, "f32"),
                                         ("RR", 8, 56, 1400, "f32"), ("STREAM_ONLY", 4, 4, 1100, "f32"),
                                         ("CM", 4, 60, 1100, "f64")):
        print(f"three steps {prec} {model} ring {ring} strip {strip} {nx}x{ny}", flush=True)
        sa, sb, (ta, tb) = run_triple(gpu, model, nx, ny, ring, strip, 7, omega, seed=13, prec=prec)
        np.testing.assert_array_equal(sa, sb)
        assert ta == tb


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_default_three_steps_with_a_two_step_tail(gpu, prec):
    # a new context on 2048 x 1024 runs three steps per launch on 24-row strips; the two steps left
    # over at the end of a call run as one two-step launch on 16-row strips (the two-step default)
    nx, ny = 2048, 1024
    rho, ux, uy = perturbed(nx, ny, 5)
    omega = inputs.rates(1e-4, "REG")
    for model in ("BGK", "K"):
        a = Sim(rho, ux, uy, prec=prec, device=gpu)
        b = Sim(rho, ux, uy, prec=prec, device=gpu)
        assert b.fusion_depth(model) == 3 and b.fusion(model) == (8, 24)
        a.set_fusion(model, 0)
        for n in (8, 5):
            a.step(model, omega, n)
            b.step(model, omega, n)
        print(f"three steps with a tail {prec} {model} {nx}x{ny}", flush=True)
        np.testing.assert_array_equal(a.state().cpu().numpy(), b.state().cpu().numpy())
        assert a.status() == b.status()
        a.close()
        b.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_raw_triples_bit_identical(gpu, prec):
    # lbm_step3_raw_many between caller buffers against single lbm_step_raw calls
    import torch

    import paper_2002_05265_amd.binding as B

    nx, ny = 131, 70
    rho, ux, uy = perturbed(nx, ny, 9)
    omega = inputs.rates(1e-4, "REG")
    for model in ("BGK", "K", "RR"):
        code = inputs.MODEL_CODES[model]
        s = Sim(rho, ux, uy, prec=prec, device=gpu)
        s.set_fusion(model, 8, 16)
        s.set_fusion_depth(model, 3)
        nb = B.lbm_state_bytes(s.ctx)
        # zero-filled, so the plane padding (never written) agrees between the two chains
        a = [torch.zeros(nb, dtype=torch.uint8, device=gpu) for _ in range(7)]
        t = [torch.zeros(nb, dtype=torch.uint8, device=gpu) for _ in range(2)]
        B.lbm_save_state(s.ctx, a[0].data_ptr())
        for k in range(6):
            B.lbm_step_raw(s.ctx, code, omega, a[k].data_ptr(), a[k + 1].data_ptr(), 5 + k)
        B.lbm_step3_raw_many(s.ctx, code, omega, [a[0].data_ptr(), t[0].data_ptr()],
                             [t[0].data_ptr(), t[1].data_ptr()], 5)
        torch.cuda.synchronize()
        print(f"raw triples {prec} {model}", flush=True)
        assert torch.equal(t[0], a[3]) and torch.equal(t[1], a[6]), (prec, model)
        with pytest.raises(LbmError):  # source and destination must differ
            B.lbm_step3_raw_many(s.ctx, code, omega, [a[0].data_ptr()], [a[0].data_ptr()], 0)
        s.set_fusion_depth(model, 2)
        with pytest.raises(LbmError) as e:  # the model no longer takes three steps per launch
            B.lbm_step3_raw_many(s.ctx, code, omega, [a[0].data_ptr()], [t[0].data_ptr()], 0)
        assert e.value.code == -2
        s.close()


def test_three_steps_blowup_step(gpu):
    # zero rates: populations only stream.  Plant A (f_1 = 5, f_3 = -4 at one node) gives a
    # negative density one step later at the left neighbour, plant B (f_3 = -0.6 two nodes right
    # of a node, f_1 = -0.6 two nodes left of it) two steps later at that node.  Started at step
    # 10 (plus one single step first for A), the first bad step falls on the first, second and
    # third step of a three-step launch; plants sit on strip and grid edges.
    nx, ny = 130, 40
    f = oracle.init_eq(4, np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    for ax, ay in ((64, 16), (0, 0), (63, 39), (129, 7)):
        a = f.copy()
        a[1, ay, ax], a[3, ay, ax] = 5.0, -4.0
        b = f.copy()
        b[3, ay, (ax + 2) % nx], b[1, ay, (ax - 2) % nx] = -0.6, -0.6
        for (g, first, want), prec in itertools.product(((a, 1, 11), (a, 0, 11), (b, 0, 12)), ("f32", "f64")):
            out = []
            for fused in (False, True):
                s = Sim(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), prec=prec, device=gpu)
                s.set_fusion("BGK", 8 if fused else 0, 16)
                if fused:
                    s.set_fusion_depth("BGK", 3)
                s.set_state(g, 10)
                s.step("BGK", [0.0] * 5, first)
                s.step("BGK", [0.0] * 5, 3)
                out.append(s.status())
                s.close()
            assert out[0] == out[1] == (13 + first, want), (ax, ay, first, prec, out)


def test_autotune_keeps_blowup_record(gpu):
    # the timed launches of autotune run ahead of the step counter through a state that turns bad
    # one step later: the blow-up record (none yet) and the state stay as they were
    nx, ny = 130, 40
    g = oracle.init_eq(4, np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    g[1, 16, 64], g[3, 16, 64] = 5.0, -4.0
    for prec in ("f32", "f64"):
        s = Sim(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), prec=prec, device=gpu)
        s.set_state(g, 10)
        before = s.state().cpu().numpy()
        s.autotune("BGK", [0.0] * 5, 1)
        assert s.status() == (10, -1), (prec, s.status())
        np.testing.assert_array_equal(s.state().cpu().numpy(), before)
        s.step("BGK", [0.0] * 5, 3)
        assert s.status() == (13, 11), (prec, s.status())
        s.close()


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_three_steps_against_oracle(gpu, prec, tol):
    nx, ny = 40, 27
    rho, ux, uy = perturbed(nx, ny, 3)
    omega = inputs.rates(1e-3, "REG")
    s = Sim(rho, ux, uy, prec=prec, device=gpu)
    s.set_fusion("CHM", 4, 8)
    s.set_fusion_depth("CHM", 3)
    s.step("CHM", omega, 9)
    got = s.state().cpu().numpy()
    s.close()
    ref = oracle.step(oracle.init_eq(4, rho, ux, uy), inputs.MODEL_CODES["CHM"], 4, omega, 9)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < tol


def test_three_steps_need_ring_4_or_8(gpu):
    # with a ring of 16 rows (or fusion off) a depth of 3 falls back to pairs (or single steps)
    nx, ny = 100, 90
    omega = inputs.rates(1e-4, "REG")
    for ring, strip in ((16, 32), (0, 0)):
        print(f"depth 3 with ring {ring}", flush=True)
        rho, ux, uy = perturbed(nx, ny, 5)
        a = Sim(rho, ux, uy, prec="f32", device=gpu)
        a.set_fusion("HM", 0)
        b = Sim(rho, ux, uy, prec="f32", device=gpu)
        b.set_fusion("HM", ring, strip)
        b.set_fusion_depth("HM", 3)
        a.step("HM", omega, 7)
        b.step("HM", omega, 7)
        np.testing.assert_array_equal(a.state().cpu().numpy(), b.state().cpu().numpy())
        assert a.status() == b.status() == (7, -1)
        a.close()
        b.close()


def test_fusion_depth_errors(gpu):
    rho, ux, uy = perturbed(32, 32, 1)
    s = Sim(rho, ux, uy, prec="f32", device=gpu)
    assert s.fusion_depth("K") == 2
    for bad in (0, 1, 4):
        with pytest.raises(LbmError):
            s.set_fusion_depth("K", bad)
    s.set_fusion_depth("K", 3)
    assert s.fusion_depth("K") == 3
    s.close()
    d = Sim(rho, ux, uy, prec="f16", device=gpu)
    with pytest.raises(LbmError):
        d.set_fusion_depth("K", 3)
    d.close()
