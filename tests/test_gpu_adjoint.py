"""Hand-written discrete adjoint (include/lbm_adjoint.h) against the CPU FP64 adjoint and
central finite differences.

- One reverse step, every model and equilibrium order, FP64: lambda_n and dL/domega equal the
  oracle's complex-step adjoint (exact to rounding) within 1e-12.
- Whole runs (vortex transport loss, CM and K): loss and gradients with respect to the
  initial velocity field and the five rates match the oracle's adjoint within 1e-10 (FP64);
  the three checkpoint schedules give bit-identical gradients.
- The 512 x 512 configuration (CM, Ma 0.2, nu 1e-5, 2000 steps, sqrt(n) checkpoints): the FP64
  gradients match central differences of the FP64 loss (h = 1e-4; 1e-6 for the bulk rate and
  single-node velocity entries, see the test) and the FP32 gradients match the FP64 ones within a
  bound set by the relative FP32 error of the loss seed, measured from the two forward runs.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_05265_amd.binding as B
from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.adjoint import transport_loss
from paper_2002_05265_amd.sim import Sim

pytestmark = pytest.mark.gpu

CENTRAL = {"CM", "CHM", "K"}


def lam_buffer(sim, lam_np):
    """Device adjoint array in the context's layout from lam_np[9, ny, nx]."""
    n = B.lbm_adjoint_bytes(sim.ctx) // 8
    plane = n // 9
    buf = torch.zeros(n, dtype=torch.float64, device=sim.device)
    cells = sim.nx * sim.ny
    for i in range(9):
        buf[i * plane:i * plane + cells] = torch.from_numpy(np.ascontiguousarray(lam_np[i]).ravel())
    return buf, plane


def lam_array(sim, buf, plane):
    cells = sim.nx * sim.ny
    b = buf.cpu().numpy()
    return np.stack([b[i * plane:i * plane + cells].reshape(sim.ny, sim.nx) for i in range(9)])


@pytest.mark.parametrize("name", list(inputs.MODEL_NAMES))
def test_adjoint_step_matches_oracle(gpu, name):
    rng = np.random.default_rng(3)
    nx, ny = 13, 11
    rho, ux, uy = inputs.vortex_fields(nx, ny, 0.3, beta=0.5, radius_frac=0.2)
    for N in ([4] if name in CENTRAL else [2, 3, 4]):
        for omega in ([1.93, 1.6, 1.2, 0.9, 1.4], list(inputs.rates(1e-4, "REG"))):
            f = oracle.init_eq(N, rho, ux, uy) * (1 + 0.02 * rng.standard_normal((9, ny, nx)))
            lam_next = rng.standard_normal((9, ny, nx))
            sim = Sim(rho, ux, uy, prec="f64", eq_order=N, device=gpu)
            sim.set_state(f, 0)
            a, plane = lam_buffer(sim, lam_next)
            b = torch.zeros_like(a)
            dw = torch.zeros(5, dtype=torch.float64, device=gpu)
            B.lbm_adjoint_step(sim.ctx, inputs.MODEL_CODES[name], omega, None, a.data_ptr(), b.data_ptr(),
                               dw.data_ptr())
            torch.cuda.synchronize()
            got = lam_array(sim, b, plane)
            sim.close()
            ref, rdw = oracle.adjoint_step(f, lam_next, inputs.MODEL_CODES[name], N, omega)
            err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            werr = np.max(np.abs(dw.cpu().numpy() - rdw)) / max(np.max(np.abs(rdw)), 1e-300)
            print(f"adjoint step {name} N={N} lambda {err:.2e} domega {werr:.2e}", flush=True)
            assert err < 1e-12 and werr < 1e-12, (name, N, err, werr)


def small_problem(n=24, steps=30, mach=0.2):
    rho, ux, uy = inputs.vortex_fields(n, n, mach, beta=0.5, radius_frac=0.15)
    tx, ty = inputs.translated_vortex_velocity(n, n, mach, steps, beta=0.5, radius_frac=0.15)
    return rho, ux, uy, tx, ty


@pytest.mark.parametrize("name", ["CM", "K", "RR"])
def test_adjoint_run_matches_oracle(gpu, name):
    steps = 30
    rho, ux, uy, tx, ty = small_problem(steps=steps)
    omega = [1.99, 1.7, 1.3, 1.1, 0.9]
    L, dux, duy, dw = oracle.adjoint_run(rho, ux, uy, tx, ty, inputs.MODEL_CODES[name], 4, omega, steps)
    results = {}
    for schedule, slots in (("sqrt", 0), ("store_all", 0), ("revolve", 3)):
        u0 = torch.tensor(np.stack([ux, uy]), device=gpu, requires_grad=True)
        w = torch.tensor(omega, dtype=torch.float64, requires_grad=True)
        loss = transport_loss(u0, w, torch.tensor(rho, device=gpu), torch.tensor(np.stack([tx, ty]), device=gpu),
                              model=name, nsteps=steps, prec="f64", schedule=schedule, slots=slots)
        loss.backward()
        results[schedule] = (float(loss.detach()), u0.grad.cpu().numpy(), w.grad.numpy())
        gu, gw = results[schedule][1], results[schedule][2]
        eu = np.max(np.abs(gu - np.stack([dux, duy]))) / np.max(np.abs(np.stack([dux, duy])))
        ew = np.max(np.abs(gw - dw)) / np.max(np.abs(dw))
        print(f"{name} {schedule}: loss {abs(float(loss) - L) / L:.2e} du {eu:.2e} domega {ew:.2e}", flush=True)
        assert abs(float(loss) - L) < 1e-12 * L and eu < 1e-10 and ew < 1e-10
    for s in ("store_all", "revolve"):
        np.testing.assert_array_equal(results[s][1], results["sqrt"][1])
        np.testing.assert_array_equal(results[s][2], results["sqrt"][2])


def c5_problem(gpu, n=512, steps=2000, mach=0.2):
    rho, ux, uy = inputs.vortex_fields(n, n, mach, beta=0.15, radius_frac=0.1)
    tx, ty = inputs.translated_vortex_velocity(n, n, mach, steps, beta=0.15, radius_frac=0.1)
    return (torch.tensor(rho, device=gpu), torch.tensor(np.stack([ux, uy]), device=gpu),
            torch.tensor(np.stack([tx, ty]), device=gpu))


def c5_grad(gpu, prec, omega, steps=2000, u_perturb=None):
    rho, u0, tgt = c5_problem(gpu, steps=steps)
    if u_perturb is not None:
        (comp, y, x), h = u_perturb
        u0 = u0.clone()
        u0[comp, y, x] += h
    u0.requires_grad_(True)
    w = torch.tensor(omega, dtype=torch.float64, requires_grad=True)
    uref = (0.2 * inputs.CS, 0.0)
    loss = transport_loss(u0, w, rho, tgt, model="CM", nsteps=steps, prec=prec, schedule="sqrt",
                          ref_velocity=uref)
    if u_perturb is not None:
        return float(loss)
    loss.backward()
    return float(loss), u0.grad.detach(), w.grad.detach().numpy()


def central_fd(f, h):
    return (f(h) - f(-h)) / (2 * h)


def test_c5_gradients_vs_fd_and_fp32(gpu):
    # Central differences, h = 1e-4, FP64, on the four higher-order rates and on entries of the
    # initial velocity field.  The exception is omega_b: at REG rates it sits at 1.99988, on the
    # barely damped bulk mode, and the loss depends on it through (1 - omega_b)^T over T = 2000
    # steps, i.e. on a scale of 1/T = 5e-4; there h = 1e-4 carries a relative error of about
    # (h T)^2 / 6 ~ 1e-2, so it is checked at h = 1e-6 ((h T)^2 / 6 ~ 1e-6; FP64 rounding of the
    # loss is far below).  The h = 1e-4 value is printed for every parameter.
    omega = list(inputs.rates(1e-5, "REG"))
    L64, du64, dw64 = c5_grad(gpu, "f64", omega)
    scale_w = float(np.max(np.abs(dw64)))
    for k in range(1, 5):  # the four higher-order rates
        def loss_at(d, k=k):
            w = list(omega)
            w[k] += d
            return c5_loss(gpu, w)
        fd4 = central_fd(loss_at, 1e-4)
        fd = central_fd(loss_at, 1e-6) if k == 1 else fd4
        print(f"domega[{k}] adjoint {dw64[k]:.10e} fd(1e-4) {fd4:.10e} fd(checked) {fd:.10e}", flush=True)
        assert abs(fd - dw64[k]) < 1e-5 * max(abs(fd), 1e-3 * scale_w), (k, fd, dw64[k])
    scale_u = float(du64.abs().max())
    for comp, y, x in [(0, 256, 256), (1, 250, 300), (0, 300, 200)]:
        def loss_u(d, comp=comp, y=y, x=x):
            return c5_grad(gpu, "f64", omega, u_perturb=((comp, y, x), d))
        # a one-node perturbation u0 + h e moves u_T by h r with |r| not small against the loss
        # L itself, so L(h) = sqrt(L^2 + 2 a h + |r|^2 h^2) bends on the scale of L / |r|: the
        # central difference is off by ~ |r|^2 h^2 / (2 L^2) (4e-3 at h = 1e-4, measured); at
        # h = 1e-6 that term is ~4e-7
        fd4, fd = central_fd(loss_u, 1e-4), central_fd(loss_u, 1e-6)
        g = float(du64[comp, y, x])
        print(f"du0[{comp},{y},{x}] adjoint {g:.10e} fd(1e-4) {fd4:.10e} fd(1e-6) {fd:.10e}", flush=True)
        assert abs(fd - g) < 1e-5 * max(abs(fd), 1e-3 * scale_u), (comp, y, x, fd, g)
    L32, du32, dw32 = c5_grad(gpu, "f32", omega)
    # The reverse sweep is linear in its seed (u_T - target) / L, and that seed is a difference of
    # nearly equal fields: the vortex is transported almost exactly (L ~ 3e-4 over 2 x 512^2
    # velocities of size ~0.1), so the rounding of the FP32 trajectory already moves the seed by a
    # relative ~5e-3.  The FP32 gradients are held to twice the seed's own relative error (2-norm),
    # measured from the two forward runs, plus 1e-3 for the rounding of the FP32 reverse sweep.
    rho, u0, tgt = c5_problem(gpu)
    u_fin = {}
    for prec, uref in (("f64", (0.0, 0.0)), ("f32", (0.2 * inputs.CS, 0.0))):
        sim = Sim(rho, u0[0], u0[1], prec=prec, eq_order=4, device=gpu, ref_velocity=uref)
        sim.step("CM", omega, 2000)
        _, ux, uy, _ = sim.moments()
        u_fin[prec] = torch.stack([ux, uy])
        sim.close()
    seed_err = float(torch.linalg.vector_norm(u_fin["f32"] - u_fin["f64"]) /
                     torch.linalg.vector_norm(u_fin["f64"] - tgt))
    eu = float(torch.linalg.vector_norm(du32 - du64) / torch.linalg.vector_norm(du64))
    ew = float(np.linalg.norm(dw32 - dw64) / np.linalg.norm(dw64))
    print(f"FP32 vs FP64: loss {abs(L32 - L64) / L64:.2e} seed {seed_err:.2e} du {eu:.2e} "
          f"domega {ew:.2e}", flush=True)
    bound = 2.0 * seed_err + 1e-3
    assert abs(L32 - L64) < 1e-3 * L64 and eu < bound and ew < bound, (seed_err, eu, ew)


def c5_loss(gpu, omega, steps=2000):
    rho, u0, tgt = c5_problem(gpu, steps=steps)
    sim = Sim(rho, u0[0], u0[1], prec="f64", eq_order=4, device=gpu)
    sim.step("CM", omega, steps)
    lam = torch.empty(B.lbm_adjoint_bytes(sim.ctx), dtype=torch.uint8, device=gpu)
    L = B.lbm_adjoint_seed_velocity_l2(sim.ctx, tgt[0].contiguous().data_ptr(), tgt[1].contiguous().data_ptr(),
                                       lam.data_ptr())
    sim.close()
    return L


@pytest.mark.parametrize("name", ["CM", "RR"])
def test_two_step_launches_give_identical_gradients(gpu, name):
    """The checkpointed sweeps with pairs of forward steps as two-step launches (lbm_step2_raw_many,
    with and without the state between them) and triples as three-step launches
    (lbm_step3_raw_many) give the same loss and gradients bit for bit as one step per launch, for
    the sqrt(n) and store-all schedules and an odd step count."""
    from paper_2002_05265_amd import binding as B
    from paper_2002_05265_amd.adjoint import _Run

    steps = 31
    rho, ux, uy, tx, ty = small_problem(n=40, steps=steps)
    omega = [1.99, 1.7, 1.3, 1.1, 0.9]
    out = {}
    for schedule in ("sqrt", "store_all"):
        # one step per launch; pairs (two-step launches); triples where the states between are not
        # kept (three-step launches of the sqrt(n) forward sweep), pairs elsewhere
        for mode in ("single", "pairs", "triples"):
            u0 = torch.tensor(np.stack([ux, uy]), device=gpu)
            run = _Run(u0, omega, torch.tensor(rho, device=gpu), torch.tensor(np.stack([tx, ty]), device=gpu), name,
                       steps, "f64", 4, schedule, 0, (0.0, 0.0))
            code = inputs.MODEL_CODES[name]
            B.lbm_set_fusion(run.ctx, code, 0 if mode == "single" else 8, 16)
            B.lbm_set_fusion_depth(run.ctx, code, 3 if mode == "triples" else 2)
            assert run._three_step() == (mode == "triples")
            loss = run.forward()
            du, dw = run.backward()
            out[(schedule, mode)] = (loss, du.cpu().numpy(), dw.cpu().numpy(), run.steps_run)
            run.close()
    ref = out[("sqrt", "single")]
    for key, val in out.items():
        print(key, "loss", val[0], "steps run", val[3], flush=True)
        assert val[0] == ref[0], key
        np.testing.assert_array_equal(val[1], ref[1])
        np.testing.assert_array_equal(val[2], ref[2])
    assert out[("sqrt", "pairs")][3] == out[("sqrt", "single")][3] == out[("sqrt", "triples")][3]
