"""Two reverse steps per launch (lbm_set_adjoint_depth(ctx, 2)): lambda_{n-1} and the rate
gradients are bit-identical to two one-step launches, in every precision and model, on grids
that span several strips with ragged edges and on the smallest grid; against the oracle's two
reverse steps within 1e-12 in FP64; pairs are taken only where the pair's output buffer is not
its input; whole checkpointed sweeps give the same loss and gradients bit for bit with one or
two reverse steps per launch."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_05265_amd.binding as B
from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.sim import Sim

pytestmark = pytest.mark.gpu

OMEGA = [1.93, 1.6, 1.2, 0.9, 1.4]
# (nx, ny): several strips across with a ragged last one, a strip height that does not divide
# ny, one strip, the smallest grid
GRIDS = [(150, 77), (64, 19), (13, 11), (2, 2)]


def adj_dtype(prec):
    return torch.float64 if prec == "f64" else torch.float32


def states_and_seed(prec, nx, ny, seed, device, eq_order=4):
    """Two raw states (after 2 and 3 forward steps of a perturbed vortex) and a random adjoint."""
    rho, ux, uy = inputs.vortex_fields(nx, ny, 0.3, beta=0.5, radius_frac=0.2)
    sim = Sim(rho, ux, uy, prec=prec, eq_order=eq_order, device=device)
    rng = np.random.default_rng(seed)
    f = oracle.init_eq(eq_order, rho, ux, uy) * (1 + 0.02 * rng.standard_normal((9, ny, nx)))
    sim.set_state(f, 0)
    sb = B.lbm_state_bytes(sim.ctx)
    st = [torch.empty(sb, dtype=torch.uint8, device=device) for _ in range(3)]
    for k in range(3):
        sim.step("BGK", OMEGA, 1)
        B.lbm_save_state(sim.ctx, st[k].data_ptr())
    n = B.lbm_adjoint_bytes(sim.ctx) // (8 if prec == "f64" else 4)
    g = torch.Generator(device="cpu").manual_seed(seed)
    lam0 = torch.randn(n, generator=g, dtype=torch.float64).to(adj_dtype(prec)).to(device)
    return sim, st, lam0


def valid(sim, buf):
    plane = buf.numel() // 9
    cells = sim.nx * sim.ny
    return torch.stack([buf[i * plane:i * plane + cells] for i in range(9)])


def run(sim, model, states, lam0, depth, nbuf):
    """lbm_adjoint_many over `states` with `nbuf` adjoint buffers in rotation; returns the final
    adjoint (valid cells) and the rate gradients."""
    B.lbm_set_adjoint_depth(sim.ctx, depth)
    bufs = [lam0.clone()] + [torch.full_like(lam0, float("nan")) for _ in range(nbuf - 1)]
    ptrs = [bufs[k % nbuf].data_ptr() for k in range(len(states) + 1)]
    dw = torch.zeros(5, dtype=torch.float64, device=lam0.device)
    B.lbm_adjoint_many(sim.ctx, inputs.MODEL_CODES[model], OMEGA, [s.data_ptr() for s in states], ptrs,
                       dw.data_ptr())
    torch.cuda.synchronize()
    return valid(sim, bufs[len(states) % nbuf]).cpu(), dw.cpu(), [valid(sim, b).cpu() for b in bufs]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("nx,ny", GRIDS)
def test_pairs_bit_identical_to_single_steps(gpu, prec, nx, ny):
    for mi, model in enumerate(inputs.MODEL_NAMES):
        sim, st, lam0 = states_and_seed(prec, nx, ny, 100 + mi, gpu)
        try:
            for count in (2, 3):
                states = [st[2], st[1], st[0]][:count]
                ref, ref_dw, _ = run(sim, model, states, lam0, 1, 3)
                got, got_dw, bufs = run(sim, model, states, lam0, 2, 3)
                assert torch.isfinite(ref).all()
                assert torch.equal(got, ref), (prec, nx, ny, model, count)
                assert torch.equal(got_dw, ref_dw), (prec, nx, ny, model, count, got_dw, ref_dw)
                # the pair's intermediate adjoint stays on chip: its buffer is not written
                assert torch.isnan(bufs[1]).all(), (prec, nx, ny, model, count)
                # two alternating buffers: the pair's output would be its input, so one step
                # per launch, every buffer written as with depth 1
                ref2, ref2_dw, _ = run(sim, model, states, lam0, 1, 2)
                got2, got2_dw, _ = run(sim, model, states, lam0, 2, 2)
                assert torch.equal(got2, ref2) and torch.equal(got2_dw, ref2_dw)
                assert torch.equal(ref2, ref)
        finally:
            sim.close()
    print(f"pairs {prec} {nx}x{ny}: all models bit-identical", flush=True)


@pytest.mark.parametrize("name", list(inputs.MODEL_NAMES))
def test_pair_matches_oracle(gpu, name):
    rng = np.random.default_rng(11)
    nx, ny = 70, 21
    rho, ux, uy = inputs.vortex_fields(nx, ny, 0.3, beta=0.5, radius_frac=0.2)
    for N in ([4] if name in ("CM", "CHM", "K") else [2, 3, 4]):
        f_n = oracle.init_eq(N, rho, ux, uy) * (1 + 0.02 * rng.standard_normal((9, ny, nx)))
        f_m = oracle.init_eq(N, rho, ux, uy) * (1 + 0.02 * rng.standard_normal((9, ny, nx)))
        lam_next = rng.standard_normal((9, ny, nx))
        sim = Sim(rho, ux, uy, prec="f64", eq_order=N, device=gpu)
        st = []
        for f in (f_n, f_m):
            sim.set_state(f, 0)
            b = torch.empty(B.lbm_state_bytes(sim.ctx), dtype=torch.uint8, device=gpu)
            B.lbm_save_state(sim.ctx, b.data_ptr())
            st.append(b)
        n = B.lbm_adjoint_bytes(sim.ctx) // 8
        plane = n // 9
        lam0 = torch.zeros(n, dtype=torch.float64, device=gpu)
        for i in range(9):
            lam0[i * plane:i * plane + nx * ny] = torch.from_numpy(lam_next[i].ravel())
        got, dw, _ = run(sim, name, st, lam0, 2, 3)
        sim.close()
        lam_n, dw1 = oracle.adjoint_step(f_n, lam_next, inputs.MODEL_CODES[name], N, OMEGA)
        ref, dw2 = oracle.adjoint_step(f_m, lam_n, inputs.MODEL_CODES[name], N, OMEGA)
        got = got.numpy().reshape(9, ny, nx)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        rdw = dw1 + dw2
        werr = np.max(np.abs(dw.numpy() - rdw)) / np.max(np.abs(rdw))
        print(f"pair {name} N={N}: lambda {err:.2e} domega {werr:.2e}", flush=True)
        assert err < 1e-12 and werr < 1e-12, (name, N, err, werr)


def test_depth_setting(gpu):
    rho, ux, uy = inputs.vortex_fields(16, 16, 0.1, beta=0.5, radius_frac=0.2)
    sim = Sim(rho, ux, uy, prec="f32", eq_order=4, device=gpu)
    try:
        assert B.lbm_get_adjoint_depth(sim.ctx) == 1
        B.lbm_set_adjoint_depth(sim.ctx, 2)
        assert B.lbm_get_adjoint_depth(sim.ctx) == 2
        for bad in (0, 3, -1):
            with pytest.raises(B.LbmError) as e:
                B.lbm_set_adjoint_depth(sim.ctx, bad)
            assert e.value.code == -1
        assert B.lbm_get_adjoint_depth(sim.ctx) == 2
    finally:
        sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sweeps_identical_with_one_or_two_reverse_steps_per_launch(gpu, prec):
    from paper_2002_05265_amd.adjoint import _Run

    steps = 31
    n = 40
    rho, ux, uy = inputs.vortex_fields(n, n, 0.2, beta=0.5, radius_frac=0.15)
    tx, ty = inputs.translated_vortex_velocity(n, n, 0.2, steps, beta=0.5, radius_frac=0.15)
    omega = [1.99, 1.7, 1.3, 1.1, 0.9]
    out = {}
    for schedule, slots in (("sqrt", 0), ("store_all", 0), ("revolve", 3)):
        for depth in (1, 2):
            u0 = torch.tensor(np.stack([ux, uy]), device=gpu)
            r = _Run(u0, omega, torch.tensor(rho, device=gpu), torch.tensor(np.stack([tx, ty]), device=gpu), "K",
                     steps, prec, 4, schedule, slots, (0.0, 0.0), reverse_depth=depth)
            loss = r.forward()
            du, dw = r.backward()
            out[(schedule, depth)] = (loss, du.cpu().numpy(), dw.cpu().numpy())
            r.close()
    ref = out[("sqrt", 1)]
    for key, val in out.items():
        print(key, "loss", val[0], "domega", val[2], flush=True)
        assert val[0] == ref[0], key
        np.testing.assert_array_equal(val[1], ref[1])
        np.testing.assert_array_equal(val[2], ref[2])
