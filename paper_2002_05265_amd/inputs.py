"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module holds none of the method's arithmetic: it only builds initial macroscopic fields
(rho, ux, uy) on the host in FP64 and draws random parameters.  Both the GPU library and the
CPU oracle receive the same arrays and compute their own equilibria from them.

Workloads (all analytic, no dataset is involved):
  * convected isothermal vortex (Section 5a: Gendre et al.'s first-order isothermal
    initialisation), centred at (L/2, L/2), node coordinates x = i, y = j;
  * double shear layer (Appendix C, Brown-Minion roll-up) with x = i / L, y = j / L;
  * uniform flow plus one random Fourier mode (random stability-sweep instances);
  * shear and acoustic plane waves (hydrodynamic-wave checks, Section 3b).
"""
from __future__ import annotations

import math

import numpy as np

CS2 = 1.0 / 3.0
CS = math.sqrt(CS2)
MODEL_NAMES = ("BGK", "RM", "HM", "CM", "CHM", "K", "PR", "RR")
MODEL_CODES = {"BGK": 0, "RM": 1, "HM": 2, "CM": 3, "CHM": 4, "K": 5, "PR": 6, "RR": 7,
               "STREAM_ONLY": 99}


def omega_nu(nu: float) -> float:
    """Relaxation frequency of the viscous moments, omega_nu = 1 / (nu / cs^2 + 1/2) (Section 4c)."""
    return 1.0 / (nu / CS2 + 0.5)


def rates(nu: float, preset: str = "SRT", omega3: float | None = None,
          omega4: float | None = None, omega_b: float | None = None) -> np.ndarray:
    """Relaxation vector (omega_nu, omega_b, omega_21, omega_12, omega_22).

    SRT: all five equal omega_nu.  REG: omega_b = omega_nu, third and fourth order equal 1
    (Section 4c).  'custom': omega3 / omega4 / omega_b given explicitly (default omega_nu)."""
    w = omega_nu(nu)
    if preset == "SRT":
        return np.array([w, w, w, w, w])
    if preset == "REG":
        return np.array([w, w, 1.0, 1.0, 1.0])
    o3 = w if omega3 is None else omega3
    o4 = w if omega4 is None else omega4
    ob = w if omega_b is None else omega_b
    return np.array([w, ob, o3, o3, o4])


def vortex_fields(nx: int, ny: int, mach: float, beta: float = 0.15, radius_frac: float = 0.1,
                  rho0: float = 1.0, center=None):
    """Convected isothermal vortex (Section 5a).

    rho = rho0 [1 - eps^2 / (2 cs^2) exp(-r^2)],
    ux  = u0 - eps (y - yc) / R exp(-r^2 / 2),  uy = eps (x - xc) / R exp(-r^2 / 2),
    eps = beta u0, u0 = Ma cs, R = radius_frac * nx (lattice units), r = |x - xc| / R.
    The displacement to the centre is taken periodically in [-L/2, L/2), which for the
    default centre (L/2, L/2) is the plain distance on the grid."""
    u0 = mach * CS
    eps = beta * u0
    R = radius_frac * nx
    xc, yc = (nx / 2.0, ny / 2.0) if center is None else center
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    dx = np.mod(x - xc + nx / 2.0, nx) - nx / 2.0
    dy = np.mod(y - yc + ny / 2.0, ny) - ny / 2.0
    r2 = (dx * dx + dy * dy) / (R * R)
    g = np.exp(-0.5 * r2)
    rho = rho0 * (1.0 - eps * eps / (2.0 * CS2) * np.exp(-r2))
    ux = u0 - eps * dy / R * g
    uy = eps * dx / R * g
    return (np.ascontiguousarray(rho), np.ascontiguousarray(np.broadcast_to(ux, (ny, nx))),
            np.ascontiguousarray(np.broadcast_to(uy, (ny, nx))))


def translated_vortex_velocity(nx: int, ny: int, mach: float, nsteps: int, beta: float = 0.15,
                               radius_frac: float = 0.1):
    """Velocity of the initial vortex translated by u0 * nsteps along x (periodic)."""
    u0 = mach * CS
    xc = np.mod(nx / 2.0 + u0 * nsteps, nx)
    _, ux, uy = vortex_fields(nx, ny, mach, beta, radius_frac, 1.0, center=(xc, ny / 2.0))
    return ux, uy


def dsl_fields(nx: int, ny: int, mach: float = 0.1, rho0: float = 1.0):
    """Double shear layer: ux = U tanh(80 (y - 1/4)) for y <= 1/2, U tanh(80 (3/4 - y)) above,
    uy = 0.05 U sin(2 pi (x + 1/4)), x = i / nx, y = j / ny, U = Ma cs, rho = rho0."""
    U = mach * CS
    x = np.arange(nx, dtype=np.float64)[None, :] / nx
    y = np.arange(ny, dtype=np.float64)[:, None] / ny
    ux = np.where(y <= 0.5, U * np.tanh(80.0 * (y - 0.25)), U * np.tanh(80.0 * (0.75 - y)))
    uy = 0.05 * U * np.sin(2.0 * np.pi * (x + 0.25))
    rho = np.full((ny, nx), rho0)
    return (rho, np.ascontiguousarray(np.broadcast_to(ux, (ny, nx))),
            np.ascontiguousarray(np.broadcast_to(uy, (ny, nx))))


def dsl_nu(nx: int, mach: float = 0.1, reynolds: float = 3.0e4) -> float:
    """Viscosity of the double shear layer at Re = U L / nu (Appendix C uses Re = 3e4)."""
    return mach * CS * nx / reynolds


def _draw_mode(rng: np.random.Generator, kmax: int):
    while True:
        kx, ky = (int(v) for v in rng.integers(-kmax, kmax + 1, size=2))
        if kx or ky:
            break
    th, ph = rng.uniform(0.0, 2.0 * np.pi, size=2)
    return kx, ky, float(th), float(ph)


def fourier_mode_fields(nx: int, ny: int, mach: float, rng: np.random.Generator,
                        amplitude: float = 1e-3, kmax: int = 4):
    """Uniform flow (Ma cs, 0) plus one velocity mode
    amplitude * (cos th, sin th) * sin(2 pi (kx i / nx + ky j / ny) + phi),
    integers kx, ky in [-kmax, kmax] not both zero, th and phi uniform in [0, 2 pi), rho = 1."""
    kx, ky, th, ph = _draw_mode(rng, kmax)
    i = np.arange(nx, dtype=np.float64)[None, :]
    j = np.arange(ny, dtype=np.float64)[:, None]
    s = np.sin(2.0 * np.pi * (kx * i / nx + ky * j / ny) + ph)
    ux = mach * CS + amplitude * np.cos(th) * s
    uy = amplitude * np.sin(th) * s
    return np.ones((ny, nx)), np.ascontiguousarray(ux), np.ascontiguousarray(uy)


def shear_wave_fields(n: int, mach: float, amplitude: float = 1e-5):
    """uy = A sin(2 pi x / n) on a mean flow (Ma cs, 0), rho = 1 (shear wave along x)."""
    x = np.arange(n, dtype=np.float64)[None, :]
    ux = np.full((n, n), mach * CS)
    uy = np.ascontiguousarray(np.broadcast_to(amplitude * np.sin(2.0 * np.pi * x / n), (n, n)))
    return np.ones((n, n)), ux, uy


def sound_wave_fields(n: int, amplitude: float = 1e-6):
    """rho = 1 + A sin(2 pi x / n), u = 0 (standing acoustic wave along x)."""
    x = np.arange(n, dtype=np.float64)[None, :]
    rho = np.ascontiguousarray(np.broadcast_to(1.0 + amplitude * np.sin(2.0 * np.pi * x / n), (n, n)))
    return rho, np.zeros((n, n)), np.zeros((n, n))


def random_cells(n: int, rng: np.random.Generator, spread: float = 0.05, umax: float = 0.15):
    """n random positive D2Q9 population vectors near a moving equilibrium shape:
    f_i = base_i (1 + 3 c_i . u) (1 + spread * N(0, 1)), base = (4/9, 1/9 x4, 1/36 x4),
    u uniform in [-umax, umax]^2, density scaled by U[0.9, 1.1]."""
    base = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
    u = rng.uniform(-umax, umax, size=(n, 2))
    shape = base[None, :] * (1.0 + 3.0 * (u[:, :1] * cx[None] + u[:, 1:] * cy[None]))
    f = shape * (1.0 + spread * rng.standard_normal((n, 9)))
    f *= rng.uniform(0.9, 1.1, size=(n, 1))
    return np.ascontiguousarray(f)


SWEEP_SIDES = (64, 96, 128, 192, 256, 384, 512)


def sweep_instances(n: int = 512, seed: int = 2002_05265, sides=SWEEP_SIDES, models=MODEL_NAMES,
                    ma_range=(0.0, 0.6), log10_nu_range=(-7.0, -2.0), preset: str = "SRT"):
    """Parameters of a random stability sweep: side ~ U(sides), Ma ~ U(ma_range),
    log10 nu ~ U(log10_nu_range), model ~ U(models), one Fourier-mode perturbation seed each."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        side = int(rng.choice(sides))
        ma = float(rng.uniform(*ma_range))
        nu = float(10.0 ** rng.uniform(*log10_nu_range))
        model = str(rng.choice(models))
        out.append({"index": k, "nx": side, "ny": side, "mach": ma, "nu": nu, "model": model,
                    "omega": rates(nu, preset), "field_seed": seed + 1 + k})
    return out


def sweep_fields(inst: dict):
    rng = np.random.default_rng(inst["field_seed"])
    return fourier_mode_fields(inst["nx"], inst["ny"], inst["mach"], rng)


def sweep_mode(inst: dict):
    """(kx, ky) of the Fourier mode of sweep_fields(inst): the fields depend on the node (i, j)
    only through the phase kx i / nx + ky j / ny."""
    kx, ky, _, _ = _draw_mode(np.random.default_rng(inst["field_seed"]), 4)
    return kx, ky


def stratified_sweep_instances(per_model: int = 2, side: int = 64, seed: int = 2002_05265 + 20_000,
                               ma_range=(0.0, 0.6), log10_nu_range=(-7.0, -2.0)):
    """A stratified subset of the random stability sweep: per_model instances of every model on
    side x side grids, Ma ~ U(ma_range), log10 nu ~ U(log10_nu_range), the SRT and REG presets in
    turn within each model, one Fourier-mode perturbation seed each."""
    rng = np.random.default_rng(seed)
    out = []
    for m, model in enumerate(MODEL_NAMES):
        for j in range(per_model):
            k = m * per_model + j
            ma = float(rng.uniform(*ma_range))
            nu = float(10.0 ** rng.uniform(*log10_nu_range))
            preset = "SRT" if j % 2 == 0 else "REG"
            out.append({"index": k, "nx": side, "ny": side, "mach": ma, "nu": nu, "model": model,
                        "preset": preset, "omega": rates(nu, preset), "eq_order": 4,
                        "field_seed": seed + 1 + k})
    return out
