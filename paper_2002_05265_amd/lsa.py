"""Linear stability analysis of the stream-and-collide scheme on the GPU (Section 4, Appendix A).

About a uniform flow (density 1, velocity U = Ma cs (cos phi, sin phi)) a plane-wave perturbation of
wave number k is multiplied every step by M(k) = diag(exp(-i xi . k)) J_C (include/lbm_lsa.h); the
scheme is linearly stable for that flow when the spectral radius of M(k) is at most one for every k.
The stability domain of Section 4c is the largest Ma, per viscosity, below which every flow direction
and every wave number is stable.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binding as B
from .inputs import CS, MODEL_CODES, rates


def point(model, nu: float, mach: float, phi: float = 0.0, preset: str = "SRT", eq_order: int = 4,
          omega=None) -> dict:
    u = mach * CS
    return {"model": MODEL_CODES[model] if isinstance(model, str) else int(model), "eq_order": eq_order,
            "omega": list(rates(nu, preset) if omega is None else omega),
            "ux": u * math.cos(phi), "uy": u * math.sin(phi)}


def k_grid(n: int, device="cuda:0"):
    """(kx, ky) flattened over an n x n grid of [-pi, pi)^2 (row-major in ky, kx)."""
    k = torch.arange(n, dtype=torch.float64, device=device) * (2.0 * math.pi / n) - math.pi
    ky, kx = torch.meshgrid(k, k, indexing="ij")
    return kx.reshape(-1).contiguous(), ky.reshape(-1).contiguous()


def jacobian(pt: dict, device="cuda:0") -> torch.Tensor:
    J = torch.empty((9, 9), dtype=torch.float64, device=device)
    B.lbm_lsa_jacobian(B.make_lsa_points([pt]), J.data_ptr(), torch.cuda.current_stream(device).cuda_stream)
    return J


def eigenvalues(pt: dict, kx: torch.Tensor, ky: torch.Tensor) -> torch.Tensor:
    """Complex (nk, 9) eigenvalues of M(k) (unordered)."""
    nk = kx.numel()
    out = torch.empty((nk, 9, 2), dtype=torch.float64, device=kx.device)
    B.lbm_lsa_eigenvalues(B.make_lsa_points([pt]), kx.data_ptr(), ky.data_ptr(), nk, out.data_ptr(),
                          torch.cuda.current_stream(kx.device).cuda_stream)
    return torch.view_as_complex(out)


def radius(points, kx: torch.Tensor, ky: torch.Tensor, chunk: int = 1 << 26) -> torch.Tensor:
    """Spectral radius (npts, nk) of M(k) for every point and wave number."""
    nk = kx.numel()
    out = torch.empty((len(points), nk), dtype=torch.float64, device=kx.device)
    per = max(1, chunk // nk)
    stream = torch.cuda.current_stream(kx.device).cuda_stream
    for a in range(0, len(points), per):
        part = points[a:a + per]
        B.lbm_lsa_radius(B.make_lsa_points(part), kx.data_ptr(), ky.data_ptr(), nk, out[a:a + len(part)].data_ptr(),
                         stream)
    return out


def dvbe_growth(points, kx: torch.Tensor, ky: torch.Tensor, tau: float = 1.0, chunk: int = 1 << 26) -> torch.Tensor:
    """Largest growth rate max Im(omega) (npts, nk) of the BGK discrete-velocity Boltzmann equation
    about each point's flow (only eq_order, ux, uy are used), for every wave number."""
    nk = kx.numel()
    out = torch.empty((len(points), nk), dtype=torch.float64, device=kx.device)
    per = max(1, chunk // nk)
    stream = torch.cuda.current_stream(kx.device).cuda_stream
    for a in range(0, len(points), per):
        part = points[a:a + per]
        B.lbm_lsa_dvbe_growth(B.make_lsa_points(part), tau, kx.data_ptr(), ky.data_ptr(), nk,
                              out[a:a + len(part)].data_ptr(), stream)
    return out


def dvbe_critical_mach(eq_order: int, phi: float, machs, kmax: float = 100.0, n: int = 64, tol: float = 1e-10,
                       device="cuda:0") -> float:
    """Largest Ma of `machs` below which (every smaller Ma included) the DVBE is linearly stable in
    flow direction phi: no wave number of a polar grid (n radii from 1e-2 to kmax, log-spaced, x n
    angles) grows faster than tol.  The growth rate is homogeneous in (k, 1/tau), so tau = 1."""
    r = torch.logspace(-2.0, math.log10(kmax), n, dtype=torch.float64, device=device)
    t = torch.arange(n, dtype=torch.float64, device=device) * (2.0 * math.pi / n)
    rr, tt = torch.meshgrid(r, t, indexing="ij")
    kx = (rr * torch.cos(tt)).reshape(-1).contiguous()
    ky = (rr * torch.sin(tt)).reshape(-1).contiguous()
    pts = [point("BGK", 0.0, ma, phi, "SRT", eq_order, omega=[1.0] * 5) for ma in machs]
    g = torch.nan_to_num(dvbe_growth(pts, kx, ky), nan=math.inf).amax(dim=1).cpu().numpy()
    best = 0.0
    for ma, gm in zip(machs, g):
        if gm > tol:
            break
        best = ma
    return best


def stability_domain(models_presets, nus, machs, phis, n: int = 64, tol: float = 1e-10, eq_order: int = 4,
                     device="cuda:0"):
    """Largest stable Ma on the grid `machs` per (model, preset, nu): every Ma up to it is stable for
    every flow direction in `phis` and every wave number of the n x n grid (max |lambda| <= 1 + tol).
    Returns (table, max radius array [model-preset, nu, Ma, phi], seconds)."""
    kx, ky = k_grid(n, device)
    pts = [point(m, nu, ma, phi, p, eq_order) for m, p in models_presets for nu in nus for ma in machs for phi in phis]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    r = radius(pts, kx, ky)
    rmax = torch.nan_to_num(r, nan=math.inf).amax(dim=1)
    e1.record()
    torch.cuda.synchronize()
    R = rmax.reshape(len(models_presets), len(nus), len(machs), len(phis)).cpu().numpy()
    stable = (R <= 1.0 + tol).all(axis=3)
    table = {}
    for a, (m, p) in enumerate(models_presets):
        for b, nu in enumerate(nus):
            best = 0.0
            for c, ma in enumerate(machs):
                if not stable[a, b, c]:
                    break
                best = ma
            table[(m, p, nu)] = best
    return table, R, e0.elapsed_time(e1) * 1e-3
