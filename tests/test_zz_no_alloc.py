"""lbm_moments_noalloc, the moments entry point for callers that cannot allocate device memory,
against lbm_moments: the same fields and totals, bit for bit (the same kernels sum in the same
order), on two calls in a row on different contexts, the second grid smaller and ragged."""
import pytest
import torch

import paper_2002_05265_amd.binding as B
from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.sim import Sim


def _noalloc(sim, device, want_fields=True):
    out = [torch.full((sim.ny, sim.nx), float("nan"), dtype=torch.float64, device=device)
           for _ in range(3)]
    tot = torch.full((6,), float("nan"), dtype=torch.float64, device=device)
    ptrs = [t.data_ptr() for t in out] if want_fields else [None, None, None]
    B.lbm_moments_noalloc(sim.ctx, *ptrs, tot.data_ptr())
    sim.stream.synchronize()
    return out, tot.cpu().tolist()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_noalloc_moments_equal_lbm_moments(gpu, prec):
    omega = inputs.rates(1e-4, "REG")
    # two calls in a row: a larger grid, then a smaller ragged one (the static partials of the
    # first call are still in the array when the second runs)
    for nx, ny, model, steps in [(320, 256, "K", 7), (67, 45, "RR", 5)]:
        print(f"noalloc: {prec} {nx}x{ny} {model} {steps} steps", flush=True)
        rho, ux, uy = inputs.vortex_fields(nx, ny, 0.2)
        sim = Sim(rho, ux, uy, prec=prec, eq_order=4, device=gpu)
        try:
            sim.step(model, omega, steps)
            out, tot = _noalloc(sim, gpu)
            r, u, v, ref_tot = sim.moments()
            torch.cuda.synchronize()
            assert torch.equal(out[0], r) and torch.equal(out[1], u) and torch.equal(out[2], v)
            assert tot == ref_tot, (tot, ref_tot)
            assert tot[5] == steps and abs(tot[0] / (nx * ny) - 1.0) < 1e-3
            # totals only (no fields), again identical
            _, tot2 = _noalloc(sim, gpu, want_fields=False)
            assert tot2 == ref_tot
        finally:
            sim.close()


@pytest.mark.gpu
def test_noalloc_moments_rejects_grids_beyond_its_scratch(gpu):
    # 4097 x 3856: 17 x 3856 = 65552 reduction blocks of 256 nodes, above the 65536 the static
    # array holds; lbm_moments still works on it
    nx, ny = 4097, 3856
    z = torch.zeros((ny, nx), dtype=torch.float64, device=gpu)
    sim = Sim(z + 1.0, z, z, prec="f16", eq_order=4, device=gpu)
    try:
        tot = torch.zeros(6, dtype=torch.float64, device=gpu)
        with pytest.raises(B.LbmError) as e:
            B.lbm_moments_noalloc(sim.ctx, None, None, None, tot.data_ptr())
        assert e.value.code == -1  # LBM_EINVAL
        assert "65536" in B.lbm_last_error()
        ref = sim.totals()
        assert abs(ref[0] / (nx * ny) - 1.0) < 1e-6
    finally:
        sim.close()
