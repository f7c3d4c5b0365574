"""FP64 CPU oracle of the D2Q9 stream-and-collide method (Coreixas et al. 2020, Appendix B).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the HIP library is
checked against.  Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it.  It shares no code with the GPU path: the arithmetic lives
in ``lbm_oracle.cpp`` (built with ``-O2 -ffp-contract=off``, single-threaded), and this module
only marshals numpy arrays.  The loss gradient and the adjoint driver below are plain numpy.

Array conventions: populations ``f[q, y, x]`` (float64, C order), scalar fields ``[y, x]``.
Velocity order i = 0..8: (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).

Parity status: every function is pinned by tests in ``tests/test_oracle_*.py`` against the
paper's closed forms, invariants and special cases; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import pathlib
import subprocess

import numpy as np

HERE = pathlib.Path(__file__).resolve().parent
LIB_PATH = HERE / "liblbm_oracle.so"
SRC_PATH = HERE / "lbm_oracle.cpp"

BGK, RM, HM, CM, CHM, K, PR, RR, STREAM_ONLY = 0, 1, 2, 3, 4, 5, 6, 7, 99
MODELS = {"BGK": BGK, "RM": RM, "HM": HM, "CM": CM, "CHM": CHM, "K": K, "PR": PR, "RR": RR}
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
CS2 = 1.0 / 3.0


def build(force: bool = False) -> pathlib.Path:
    """Compile the oracle shared library with g++ (plain, -O2, no FP contraction)."""
    if LIB_PATH.exists() and not force:
        return LIB_PATH
    tmp = LIB_PATH.with_suffix(".so.tmp")
    cmd = ["g++", "-O2", "-ffp-contract=off", "-std=c++17", "-fPIC", "-shared",
           str(SRC_PATH), "-o", str(tmp)]
    subprocess.run(cmd, check=True)
    tmp.replace(LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            build()
        L = ctypes.CDLL(str(LIB_PATH))
        dp = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        L.oracle_collide_cell.argtypes = [i, i, dp, dp, dp]
        L.oracle_feq_cell.argtypes = [i, d, d, d, dp]
        L.oracle_feq_cell.restype = None
        L.oracle_moments_cell.argtypes = [i, dp, dp]
        L.oracle_moments_cell.restype = None
        L.oracle_init_eq.argtypes = [i, i, i, dp, dp, dp, dp]
        L.oracle_init_eq.restype = None
        L.oracle_step.argtypes = [i, i, i, i, dp, dp, i]
        L.oracle_moments.argtypes = [i, i, dp, dp, dp, dp, dp]
        L.oracle_moments.restype = None
        L.oracle_collide_jacobian.argtypes = [i, i, dp, dp, dp, dp]
        L.oracle_feq_jacobian.argtypes = [i, d, d, d, dp]
        L.oracle_feq_jacobian.restype = None
        L.oracle_adjoint_step.argtypes = [i, i, i, i, dp, dp, dp, dp, dp]
        L.oracle_feq_vjp.argtypes = [i, i, i, dp, dp, dp, dp, dp, dp]
        L.oracle_feq_vjp.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def collide_cell(model: int, N: int, omega, f) -> np.ndarray:
    """Post-collision populations of one cell (Appendix B)."""
    w, f = _f64(omega), _f64(f)
    out = np.empty(9)
    _check(lib().oracle_collide_cell(model, N, _p(w), _p(f), _p(out)), "collide")
    return out


def feq_cell(N: int, rho: float, ux: float, uy: float) -> np.ndarray:
    """Discrete equilibrium of order N (eq. extendedFeq)."""
    out = np.empty(9)
    lib().oracle_feq_cell(N, rho, ux, uy, _p(out))
    return out


def moments_cell(kind: str, f) -> np.ndarray:
    """3x3 moments X[p, q] of one cell: kind in raw / hermite / central / central_hermite."""
    k = {"raw": 0, "hermite": 1, "central": 2, "central_hermite": 3}[kind]
    out = np.empty(9)
    lib().oracle_moments_cell(k, _p(_f64(f)), _p(out))
    return out.reshape(3, 3)


def init_eq(N: int, rho, ux, uy) -> np.ndarray:
    rho, ux, uy = _f64(rho), _f64(ux), _f64(uy)
    ny, nx = rho.shape
    f = np.empty((9, ny, nx))
    lib().oracle_init_eq(nx, ny, N, _p(rho), _p(ux), _p(uy), _p(f))
    return f


def step(f, model: int, N: int, omega, nsteps: int) -> np.ndarray:
    """Return the state after nsteps of collide-then-stream (input is not modified)."""
    g = np.array(f, dtype=np.float64, order="C", copy=True)
    _, ny, nx = g.shape
    w = _f64(omega)
    _check(lib().oracle_step(nx, ny, model, N, _p(w), _p(g), nsteps), "step")
    return g


def moments(f):
    """(rho, ux, uy, totals) with totals = [sum rho, sum rho ux, sum rho uy, sum rho u^2/2, mean u^2]."""
    f = _f64(f)
    _, ny, nx = f.shape
    rho, ux, uy, tot = np.empty((ny, nx)), np.empty((ny, nx)), np.empty((ny, nx)), np.empty(5)
    lib().oracle_moments(nx, ny, _p(f), _p(rho), _p(ux), _p(uy), _p(tot))
    return rho, ux, uy, tot


def collide_jacobian(model: int, N: int, omega, f):
    """(J, Jw): J[i, j] = dC_i/df_j, Jw[i, k] = dC_i/domega_k (complex-step, exact to rounding)."""
    J, Jw = np.empty(81), np.empty(45)
    _check(lib().oracle_collide_jacobian(model, N, _p(_f64(omega)), _p(_f64(f)), _p(J), _p(Jw)),
           "jacobian")
    return J.reshape(9, 9), Jw.reshape(9, 5)


def feq_jacobian(N: int, rho: float, ux: float, uy: float) -> np.ndarray:
    d = np.empty(18)
    lib().oracle_feq_jacobian(N, rho, ux, uy, _p(d))
    return d.reshape(9, 2)


def adjoint_step(f_n, lam_next, model: int, N: int, omega):
    """(lam_n, domega) of one reverse step of f_{n+1} = S C(f_n)."""
    f_n, lam_next = _f64(f_n), _f64(lam_next)
    _, ny, nx = f_n.shape
    lam = np.empty_like(f_n)
    dw = np.zeros(5)
    _check(lib().oracle_adjoint_step(nx, ny, model, N, _p(_f64(omega)), _p(f_n), _p(lam_next),
                                     _p(lam), _p(dw)), "adjoint step")
    return lam, dw


def feq_vjp(N: int, rho, ux, uy, lam0):
    rho, ux, uy, lam0 = _f64(rho), _f64(ux), _f64(uy), _f64(lam0)
    ny, nx = rho.shape
    dux, duy = np.empty((ny, nx)), np.empty((ny, nx))
    lib().oracle_feq_vjp(nx, ny, N, _p(rho), _p(ux), _p(uy), _p(lam0), _p(dux), _p(duy))
    return dux, duy


def velocity_loss(f, ux_t, uy_t):
    """L = || u(f) - u_target ||_2 over all nodes and both components, and dL/df."""
    f = _f64(f)
    rho = f.sum(axis=0)
    ux = np.tensordot(CX.astype(float), f, axes=1) / rho
    uy = np.tensordot(CY.astype(float), f, axes=1) / rho
    ex, ey = ux - ux_t, uy - uy_t
    L = float(np.sqrt(np.sum(ex * ex) + np.sum(ey * ey)))
    gx, gy = ex / L, ey / L
    # du_a/df_i = (c_ia - u_a) / rho
    lam = ((CX[:, None, None] - ux[None]) * gx[None] + (CY[:, None, None] - uy[None]) * gy[None]) / rho[None]
    return L, lam


def adjoint_run(rho0, ux0, uy0, ux_t, uy_t, model: int, N: int, omega, nsteps: int):
    """Loss and gradients (dL/dux0, dL/duy0, dL/domega) of
    L = || u(f_T) - u_target ||_2,  f_{n+1} = S C(f_n; omega),  f_0 = f^eq_N(rho0, u0).
    Forward states are all kept in memory (small grids only)."""
    states = [init_eq(N, rho0, ux0, uy0)]
    for _ in range(nsteps):
        states.append(step(states[-1], model, N, omega, 1))
    L, lam = velocity_loss(states[-1], ux_t, uy_t)
    dw = np.zeros(5)
    for n in range(nsteps - 1, -1, -1):
        lam, d = adjoint_step(states[n], lam, model, N, omega)
        dw += d
    dux, duy = feq_vjp(N, rho0, ux0, uy0, lam)
    return L, dux, duy, dw


def forward_loss(rho0, ux0, uy0, ux_t, uy_t, model: int, N: int, omega, nsteps: int) -> float:
    f = step(init_eq(N, rho0, ux0, uy0), model, N, omega, nsteps)
    return velocity_loss(f, ux_t, uy_t)[0]


# ---------------------------------------------------------------------------------------------
# Linear stability analysis (Section 4, Appendix A), built from the collision Jacobian above and
# a library eigenvalue routine.

def velocities():
    """(cx, cy) of the nine lattice velocities in the oracle's order."""
    cx, cy = (ctypes.c_int * 9)(), (ctypes.c_int * 9)()
    lib().oracle_velocities(cx, cy)
    return np.array(cx[:], dtype=np.float64), np.array(cy[:], dtype=np.float64)


def lsa_jacobian(model: int, N: int, omega, ux: float, uy: float) -> np.ndarray:
    """delta + J of eq. DiscretePerturbedEq: d f*_i / d f_j at the uniform flow f = f^eq_N(1, U)."""
    return collide_jacobian(model, N, omega, feq_cell(N, 1.0, ux, uy))[0]


def lsa_matrix(J: np.ndarray, kx: float, ky: float) -> np.ndarray:
    """M^D(k) = E^D (delta + J), E^D = diag(exp(-i xi_i . k)) (Appendix A, eigenvalue problem)."""
    cx, cy = velocities()
    return np.exp(-1j * (cx * kx + cy * ky))[:, None] * J


def lsa_eigenvalues(J: np.ndarray, kx: float, ky: float) -> np.ndarray:
    """Eigenvalues exp(-i omega) of M^D(k); the growth rate of each wave is log |lambda|."""
    return np.linalg.eigvals(lsa_matrix(J, kx, ky))


def dvbe_matrix(N: int, tau: float, ux: float, uy: float, kx: float, ky: float) -> np.ndarray:
    """M^C = E^C + i J^C of the BGK discrete-velocity Boltzmann equation (Appendix A), with
    E^C = diag(xi_i . k) and J^C = -(I - F) / tau, F = d f^eq / d f at f^eq_N(1, U).  F is the
    Jacobian of the BGK collision at omega = 1 (whose post-collision state is f^eq itself)."""
    cx, cy = velocities()
    F = lsa_jacobian(BGK, N, [1.0] * 5, ux, uy)
    return np.diag(cx * kx + cy * ky) + 1j * (-(np.eye(9) - F) / tau)
