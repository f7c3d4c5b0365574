"""Parity at the benchmark's full size and launch configuration (4096 x 4096 double shear
layer, the same Sim / lbm_step path bench.py times: a new context's default of three steps per
launch in FP32 and FP64, here one such launch and then a two-step one; two steps per launch in
FP16 storage), on sampled nodes.

After k steps a node depends only on nodes within distance k (one lattice link per step), so
the oracle recomputes a sampled node exactly from a (2k + 3)^2 patch of the analytic initial
fields: the patch is run periodically and its wrap-around errors cannot reach the centre in k
steps.  Samples include the four corners and edge nodes so the periodic wrap of the full grid
is covered.  Global invariants (mass and momentum) are checked over the whole grid.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.sim import Sim

pytestmark = pytest.mark.gpu

N = 4096
STEPS = 5


def sample_nodes(rng, n, count=48):
    pts = [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (0, n // 2), (n // 2, 0),
           (n - 1, n // 3), (n // 3, n - 1), (n // 4, n // 4 + 1)]
    pts += [(int(a), int(b)) for a, b in rng.integers(0, n, size=(count, 2))]
    return pts


def patch_reference(fields, y, x, model, omega, steps):
    rho, ux, uy = fields
    r = steps + 1
    ys = (np.arange(y - r, y + r + 1)) % rho.shape[0]
    xs = (np.arange(x - r, x + r + 1)) % rho.shape[1]
    sub = [a[np.ix_(ys, xs)] for a in (rho, ux, uy)]
    f = oracle.init_eq(4, *sub)
    f = oracle.step(f, inputs.MODEL_CODES[model], 4, omega, steps)
    return f[:, r, r]


def fp16_bound(ref, steps):
    """Error bound of binary16 storage: every stored deviation h = f - w_i (the reference state
    is rho0 = 1 at rest) is rounded to nearest with relative error <= 2^-11 each step, and a
    population written by a step is a near-identity combination of the node's nine pulled values,
    so each step adds at most the nine roundings of a node, 9 * 2^-11 * max|h|: after `steps`
    steps |f - f_oracle| <= 9 * steps * 2^-11 * max|h| (max|h| over the samples).  A dropped term
    or wrong index moves f by O(|h|), far above it."""
    one, zero = np.ones((1, 1)), np.zeros((1, 1))
    w = oracle.init_eq(4, one, zero, zero)[:, 0, 0]  # f^eq(1, 0): the stored reference
    h = np.abs(ref - w[:, None])
    return 9 * steps * 2.0 ** -11 * float(h.max())


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-12), ("f16", None)])
def test_fullsize_sampled(gpu, prec, tol):
    fields = inputs.dsl_fields(N, N, 0.1)
    omega = inputs.rates(inputs.dsl_nu(N), "REG")
    rng = np.random.default_rng(4096)
    nodes = sample_nodes(rng, N)
    iy = torch.tensor([p[0] for p in nodes], device=gpu)
    ix = torch.tensor([p[1] for p in nodes], device=gpu)
    for model in inputs.MODEL_NAMES:
        print(f"full size {prec} {model}", flush=True)
        sim = Sim(*fields, prec=prec, eq_order=4, device=gpu)
        # the kernel timed at this size: three steps per launch (FP16: two)
        assert sim.fusion(model)[0] > 0 and sim.fusion_depth(model) == (2 if prec == "f16" else 3)
        t0 = sim.totals()
        sim.step(model, omega, STEPS)
        state = sim.state()
        got = state[:, iy, ix].cpu().numpy()
        del state
        t1 = sim.totals()
        sim.close()
        torch.cuda.empty_cache()
        ref = np.stack([patch_reference(fields, y, x, model, omega, STEPS) for y, x in nodes], axis=1)
        if prec == "f16":
            err = float(np.max(np.abs(got - ref)))
            bound = fp16_bound(ref, STEPS)
            print(f"  f16 {model}: max |f - f_oracle| {err:.3e}, bound {bound:.3e}", flush=True)
            assert err < bound, (model, err, bound)
        else:
            err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
            assert err < tol, (model, prec, err)
        # mass and momentum are conserved over the whole grid: up to the FP64 sums in FP64 and the
        # stored roundings in FP32; in FP16 each stored value moves a node's mass by up to
        # 2^-11 |h|, and on this field (u depends on y alone in one component, on x alone in the
        # other) equal values round alike, so the roundings add up coherently rather than cancel:
        # the per-node bound of fp16_bound, times the nodes
        mass_tol = {"f64": 1e-13, "f32": 1e-7}[prec] if prec != "f16" else fp16_bound(ref, STEPS)
        assert abs(t1[0] - t0[0]) < mass_tol * t0[0], (t0[0], t1[0])
        assert abs(t1[1] - t0[1]) < mass_tol * t0[0] and abs(t1[2] - t0[2]) < mass_tol * t0[0]
        assert t1[5] == STEPS
