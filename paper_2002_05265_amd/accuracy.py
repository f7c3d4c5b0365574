"""Long-distance transport accuracy of the collision models (Section 5d), on the batched kernel.

The convected vortex of Section 5a (beta = 0.5, R = L / 20, mean flow u0 = Ma cs along x) is run for
M convective times t_c = L / u0.  After a whole number of domain crossings a vortex transported
exactly is back where it started, so the state at M t_c is compared with the initial one through the
vorticity w = d(uy)/dx - d(ux)/dy (periodic central differences):
  - l2: ||w(T) - w(0)||_2 / ||w(0)||_2 (total error),
  - peak: max w(T) / max w(0) (dissipation of the core),
  - shift: displacement of the centroid of the positive vorticity beyond the exact transport, in
    nodes (dispersion / phase).
"""
from __future__ import annotations

import torch

from . import inputs
from .batch import Batch


def vorticity(ux: torch.Tensor, uy: torch.Tensor) -> torch.Tensor:
    """w = d(uy)/dx - d(ux)/dy with second-order central differences on the periodic grid [y][x]."""
    return 0.5 * (torch.roll(uy, -1, 1) - torch.roll(uy, 1, 1)) - 0.5 * (torch.roll(ux, -1, 0) - torch.roll(ux, 1, 0))


def velocity(f: torch.Tensor):
    """(ux, uy) of populations f[9][y][x] (D2Q9 order: rest, +x, +y, -x, -y, then the diagonals
    (+,+), (-,+), (-,-), (+,-))."""
    rho = f.sum(0)
    jx = f[1] + f[5] + f[8] - f[3] - f[6] - f[7]
    jy = f[2] + f[5] + f[6] - f[4] - f[7] - f[8]
    return jx / rho, jy / rho


def centroid(w: torch.Tensor):
    """Centroid (x, y) of the positive part of w, in node units (the vortex sits far from the edges)."""
    wp = torch.clamp(w, min=0.0)
    ny, nx = w.shape
    xs = torch.arange(nx, dtype=w.dtype, device=w.device)
    ys = torch.arange(ny, dtype=w.dtype, device=w.device)
    tot = wp.sum()
    return float((wp.sum(0) * xs).sum() / tot), float((wp.sum(1) * ys).sum() / tot)


def transport_accuracy(models_presets, Ls, mach: float = 0.5, nu: float = 1e-4, M: int = 50,
                       beta: float = 0.5, radius_frac: float = 0.05, prec: str = "f64", device="cuda:0"):
    """Run every (model, preset) at every L for M t_c; returns ({(model, preset, L): metrics},
    {L: (seconds, node updates)}).  M must be a whole number of crossings: the step count is
    M L / u0 rounded to the nearest step, and the remaining sub-step offset is reported."""
    dev = torch.device(device)
    u0 = mach * inputs.CS
    out, timing = {}, {}
    for L in Ls:
        insts = [{"nx": L, "ny": L, "model": m, "preset": p, "eq_order": 4, "omega": inputs.rates(nu, p)}
                 for m, p in models_presets]
        fields = inputs.vortex_fields(L, L, mach, beta=beta, radius_frac=radius_frac)
        steps = int(round(M * L / u0))
        b = Batch(insts, [fields] * len(insts), prec=prec, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.run(steps)
        e1.record()
        torch.cuda.synchronize()
        timing[L] = (e0.elapsed_time(e1) * 1e-3, float(steps) * L * L * len(insts))
        w0 = vorticity(torch.tensor(fields[1], device=dev), torch.tensor(fields[2], device=dev))
        c0 = centroid(w0)
        for j, (m, p) in enumerate(models_presets):
            w = vorticity(*velocity(b.state(j)))
            c = centroid(w)
            out[(m, p, L)] = {
                "l2": float(torch.linalg.vector_norm(w - w0) / torch.linalg.vector_norm(w0)),
                "peak": float(w.max() / w0.max()),
                # displacement beyond the exact transport of the rounded step count
                "shift": (c[0] - c0[0] - (steps * u0 - M * L), c[1] - c0[1]),
                "steps": steps,
                "offset_nodes": steps * u0 - M * L,
                "w": w,
            }
        _, blow = b.status()
        for j, (m, p) in enumerate(models_presets):
            out[(m, p, L)]["blowup"] = blow[j]
        b.close()
    return out, timing
