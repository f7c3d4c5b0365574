"""ctypes binding of liblbm.so (the C ABI in include/lbm.h).

Argument marshalling only: every function has the C name and forwards plain integers, floats
and pointers.  Device pointers are passed as Python ints (for example ``tensor.data_ptr()``).
A non-zero status raises :class:`LbmError` carrying the library's message.  There is no
fallback: if the HIP library is not built, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import pathlib

LIB_PATH = pathlib.Path(__file__).resolve().with_name("liblbm.so")

LBM_Q = 9
LBM_NOMEGA = 5
LBM_BGK, LBM_RM, LBM_HM, LBM_CM, LBM_CHM, LBM_K, LBM_PR, LBM_RR = range(8)
LBM_STREAM_ONLY = 99
LBM_F64, LBM_F32_SHIFTED, LBM_F16_SHIFTED = 0, 1, 2
PRECISIONS = {"f64": LBM_F64, "f32": LBM_F32_SHIFTED, "f16": LBM_F16_SHIFTED}
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_EUNSUPPORTED", -3: "LBM_EHIP", -4: "LBM_ESTATE"}

# every symbol declared in include/*.h
EXPORTS = (
    "lbm_population_bytes", "lbm_init", "lbm_init_shifted", "lbm_step", "lbm_moments", "lbm_moments_noalloc",
    "lbm_status",
    "lbm_get_state", "lbm_set_state", "lbm_set_launch", "lbm_set_fusion", "lbm_get_fusion",
    "lbm_set_fusion_depth", "lbm_get_fusion_depth", "lbm_autotune", "lbm_destroy", "lbm_last_error",
    "lbm_batch_population_bytes", "lbm_batch_create", "lbm_batch_run", "lbm_batch_status",
    "lbm_batch_get_state", "lbm_batch_mean_u2", "lbm_batch_set_active", "lbm_batch_rebalance",
    "lbm_batch_set_launch", "lbm_batch_set_fusion", "lbm_batch_get_fusion",
    "lbm_batch_set_fusion_depth", "lbm_batch_get_fusion_depth",
    "lbm_batch_autotune", "lbm_batch_residency", "lbm_batch_destroy",
    "lbm_state_bytes", "lbm_adjoint_bytes", "lbm_save_state", "lbm_load_state", "lbm_step_raw",
    "lbm_step_raw_many", "lbm_step2_raw_many", "lbm_step3_raw_many", "lbm_adjoint_many", "lbm_adjoint_flush",
    "lbm_set_adjoint_depth", "lbm_get_adjoint_depth",
    "lbm_adjoint_seed_velocity_l2", "lbm_adjoint_step", "lbm_eq_vjp",
    "lbm_lsa_jacobian", "lbm_lsa_eigenvalues", "lbm_lsa_radius", "lbm_lsa_dvbe_growth",
)


class InstanceDesc(ctypes.Structure):
    """lbm_instance_desc (include/lbm_batch.h)."""
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("model", ctypes.c_int),
                ("eq_order", ctypes.c_int), ("omega", ctypes.c_double * 5), ("rho0", ctypes.c_double),
                ("ux0", ctypes.c_double), ("uy0", ctypes.c_double)]


class LsaPoint(ctypes.Structure):
    """lbm_lsa_point (include/lbm_lsa.h)."""
    _fields_ = [("model", ctypes.c_int), ("eq_order", ctypes.c_int), ("omega", ctypes.c_double * 5),
                ("ux", ctypes.c_double), ("uy", ctypes.c_double)]


class LbmError(RuntimeError):
    def __init__(self, code: int, what: str, message: str):
        super().__init__(f"{what}: {STATUS.get(code, code)}: {message}")
        self.code = code


_lib = None
_vp, _i, _d, _sz, _ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_longlong
_dp = ctypes.POINTER(ctypes.c_double)


def _declare(L: ctypes.CDLL):
    sig = {
        "lbm_population_bytes": (_sz, [_i, _i, _i]),
        "lbm_init": (_i, [ctypes.POINTER(_vp), _i, _i, _i, _i, _d, _vp, _vp, _vp, _vp, _sz, _vp]),
        "lbm_init_shifted": (_i, [ctypes.POINTER(_vp), _i, _i, _i, _i, _d, _d, _d, _vp, _vp, _vp, _vp,
                                  _sz, _vp]),
        "lbm_step": (_i, [_vp, _i, _dp, _i]),
        "lbm_moments": (_i, [_vp, _vp, _vp, _vp, _dp]),
        "lbm_moments_noalloc": (_i, [_vp, _vp, _vp, _vp, _vp]),
        "lbm_status": (_i, [_vp, ctypes.POINTER(_ll), ctypes.POINTER(_ll)]),
        "lbm_get_state": (_i, [_vp, _vp]),
        "lbm_set_state": (_i, [_vp, _vp, _ll]),
        "lbm_set_launch": (_i, [_vp, _i, _i, _i]),
        "lbm_set_fusion": (_i, [_vp, _i, _i, _i]),
        "lbm_get_fusion": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
        "lbm_set_fusion_depth": (_i, [_vp, _i, _i]),
        "lbm_get_fusion_depth": (_i, [_vp, _i, ctypes.POINTER(_i)]),
        "lbm_autotune": (_i, [_vp, _i, _dp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), _dp]),
        "lbm_destroy": (None, [_vp]),
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_batch_population_bytes": (_sz, [ctypes.POINTER(InstanceDesc), _i, _i]),
        "lbm_batch_create": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(InstanceDesc), _i, _i, _vp, _vp,
                                  _vp, _vp, _sz, _vp]),
        "lbm_batch_run": (_i, [_vp, _i]),
        "lbm_batch_status": (_i, [_vp, ctypes.POINTER(_ll), ctypes.POINTER(_ll)]),
        "lbm_batch_get_state": (_i, [_vp, _i, _vp]),
        "lbm_batch_mean_u2": (_i, [_vp, _vp]),
        "lbm_batch_set_active": (_i, [_vp, _vp]),
        "lbm_batch_rebalance": (_i, [_vp]),
        "lbm_lsa_jacobian": (_i, [_vp, _i, _vp, _vp]),
        "lbm_lsa_eigenvalues": (_i, [_vp, _vp, _vp, _i, _vp, _vp]),
        "lbm_lsa_radius": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp]),
        "lbm_lsa_dvbe_growth": (_i, [_vp, _i, _d, _vp, _vp, _i, _vp, _vp]),
        "lbm_batch_set_launch": (_i, [_vp, _i, _i]),
        "lbm_batch_set_fusion": (_i, [_vp, _i]),
        "lbm_batch_get_fusion": (_i, [_vp, ctypes.POINTER(_i)]),
        "lbm_batch_set_fusion_depth": (_i, [_vp, _i]),
        "lbm_batch_get_fusion_depth": (_i, [_vp, ctypes.POINTER(_i)]),
        "lbm_batch_autotune": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), _dp]),
        "lbm_batch_destroy": (None, [_vp]),
        "lbm_batch_residency": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
        "lbm_state_bytes": (_sz, [_vp]),
        "lbm_adjoint_bytes": (_sz, [_vp]),
        "lbm_save_state": (_i, [_vp, _vp]),
        "lbm_load_state": (_i, [_vp, _vp, _ll]),
        "lbm_step_raw": (_i, [_vp, _i, _dp, _vp, _vp, _ll]),
        "lbm_step_raw_many": (_i, [_vp, _i, _dp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i, _ll]),
        "lbm_step2_raw_many": (_i, [_vp, _i, _dp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i,
                                    _ll]),
        "lbm_step3_raw_many": (_i, [_vp, _i, _dp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i, _ll]),
        "lbm_adjoint_many": (_i, [_vp, _i, _dp, ctypes.POINTER(_vp), _i, ctypes.POINTER(_vp), _vp]),
        "lbm_adjoint_flush": (_i, [_vp, _vp]),
        "lbm_set_adjoint_depth": (_i, [_vp, _i]),
        "lbm_get_adjoint_depth": (_i, [_vp, ctypes.POINTER(_i)]),
        "lbm_adjoint_seed_velocity_l2": (_i, [_vp, _vp, _vp, _vp, _dp]),
        "lbm_adjoint_step": (_i, [_vp, _i, _dp, _vp, _vp, _vp, _vp]),
        "lbm_eq_vjp": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    for name, (res, args) in EXTRA_SIGNATURES.items():
        if hasattr(L, name):
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args


EXTRA_SIGNATURES: dict = {}


def lib() -> ctypes.CDLL:
    """Load liblbm.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(str(LIB_PATH))
        _declare(L)
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise LbmError(rc, what, lib().lbm_last_error().decode(errors="replace"))


def _omega(omega):
    w = [float(v) for v in omega]
    if len(w) != LBM_NOMEGA:
        raise ValueError(f"omega must have {LBM_NOMEGA} entries")
    return (ctypes.c_double * LBM_NOMEGA)(*w)


def lbm_population_bytes(nx: int, ny: int, prec: int) -> int:
    return int(lib().lbm_population_bytes(nx, ny, prec))


def lbm_init(nx: int, ny: int, prec: int, eq_order: int, rho0: float, rho: int, ux: int, uy: int,
             pop_buf: int, pop_bytes: int, stream: int) -> int:
    ctx = _vp()
    _check(lib().lbm_init(ctypes.byref(ctx), nx, ny, prec, eq_order, rho0, rho, ux, uy, pop_buf,
                          pop_bytes, stream or None), "lbm_init")
    return ctx.value


def lbm_init_shifted(nx: int, ny: int, prec: int, eq_order: int, rho0: float, ux0: float, uy0: float,
                     rho: int, ux: int, uy: int, pop_buf: int, pop_bytes: int, stream: int) -> int:
    ctx = _vp()
    _check(lib().lbm_init_shifted(ctypes.byref(ctx), nx, ny, prec, eq_order, rho0, ux0, uy0, rho, ux,
                                  uy, pop_buf, pop_bytes, stream or None), "lbm_init_shifted")
    return ctx.value


def lbm_step(ctx: int, model: int, omega, nsteps: int):
    _check(lib().lbm_step(ctx, model, _omega(omega), nsteps), "lbm_step")


def lbm_moments(ctx: int, rho: int | None, ux: int | None, uy: int | None, want_totals=True):
    tot = (ctypes.c_double * 6)() if want_totals else None
    _check(lib().lbm_moments(ctx, rho, ux, uy, tot), "lbm_moments")
    return list(tot) if want_totals else None


def lbm_moments_noalloc(ctx: int, rho: int | None, ux: int | None, uy: int | None, totals: int | None):
    """totals: device address of 6 doubles (or None); nothing is synchronised or allocated."""
    _check(lib().lbm_moments_noalloc(ctx, rho, ux, uy, totals), "lbm_moments_noalloc")


def lbm_status(ctx: int):
    step, blow = _ll(), _ll()
    _check(lib().lbm_status(ctx, ctypes.byref(step), ctypes.byref(blow)), "lbm_status")
    return step.value, blow.value


def lbm_get_state(ctx: int, f: int):
    _check(lib().lbm_get_state(ctx, f), "lbm_get_state")


def lbm_set_state(ctx: int, f: int, step: int):
    _check(lib().lbm_set_state(ctx, f, step), "lbm_set_state")


def lbm_set_launch(ctx: int, model: int, rows: int, xcd: int):
    _check(lib().lbm_set_launch(ctx, model, rows, xcd), "lbm_set_launch")


def lbm_set_fusion(ctx: int, model: int, ring_rows: int, strip_rows: int):
    _check(lib().lbm_set_fusion(ctx, model, ring_rows, strip_rows), "lbm_set_fusion")


def lbm_set_fusion_depth(ctx: int, model: int, steps: int):
    _check(lib().lbm_set_fusion_depth(ctx, model, steps), "lbm_set_fusion_depth")


def lbm_get_fusion_depth(ctx: int, model: int) -> int:
    steps = _i(0)
    _check(lib().lbm_get_fusion_depth(ctx, model, ctypes.byref(steps)), "lbm_get_fusion_depth")
    return steps.value


def lbm_get_fusion(ctx: int, model: int):
    ring, strip = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().lbm_get_fusion(ctx, model, ctypes.byref(ring), ctypes.byref(strip)), "lbm_get_fusion")
    return ring.value, strip.value


def lbm_autotune(ctx: int, model: int, omega, trials: int):
    rows, xcd, us = _i(), _i(), _d()
    _check(lib().lbm_autotune(ctx, model, _omega(omega), trials, ctypes.byref(rows),
                              ctypes.byref(xcd), ctypes.byref(us)), "lbm_autotune")
    return rows.value, xcd.value, us.value


def lbm_destroy(ctx: int):
    lib().lbm_destroy(ctx)


def make_descs(descs) -> ctypes.Array:
    """Array of InstanceDesc from dicts with nx, ny, model (code), eq_order, omega, rho0."""
    arr = (InstanceDesc * len(descs))()
    for a, d in zip(arr, descs):
        a.nx, a.ny, a.model, a.eq_order = int(d["nx"]), int(d["ny"]), int(d["model"]), int(d["eq_order"])
        for k in range(5):
            a.omega[k] = float(d["omega"][k])
        a.rho0 = float(d.get("rho0", 1.0))
        a.ux0 = float(d.get("ux0", 0.0))
        a.uy0 = float(d.get("uy0", 0.0))
    return arr


def lbm_batch_population_bytes(descs: ctypes.Array, prec: int) -> int:
    return int(lib().lbm_batch_population_bytes(descs, len(descs), prec))


def lbm_batch_create(descs: ctypes.Array, prec: int, rho: int, ux: int, uy: int, pop_buf: int,
                     pop_bytes: int, stream: int) -> int:
    b = _vp()
    _check(lib().lbm_batch_create(ctypes.byref(b), descs, len(descs), prec, rho, ux, uy, pop_buf,
                                  pop_bytes, stream or None), "lbm_batch_create")
    return b.value


def lbm_batch_run(b: int, nsteps: int):
    _check(lib().lbm_batch_run(b, nsteps), "lbm_batch_run")


def lbm_batch_status(b: int, n: int):
    step = _ll()
    blow = (_ll * n)()
    _check(lib().lbm_batch_status(b, ctypes.byref(step), blow), "lbm_batch_status")
    return step.value, list(blow)


def lbm_batch_get_state(b: int, instance: int, f: int):
    _check(lib().lbm_batch_get_state(b, instance, f), "lbm_batch_get_state")


def lbm_batch_mean_u2(b: int, mean_u2: int):
    _check(lib().lbm_batch_mean_u2(b, mean_u2), "lbm_batch_mean_u2")


def lbm_batch_set_active(b: int, active: int):
    _check(lib().lbm_batch_set_active(b, active), "lbm_batch_set_active")


def lbm_batch_rebalance(b: int):
    _check(lib().lbm_batch_rebalance(b), "lbm_batch_rebalance")


def lbm_batch_set_launch(b: int, nodes_per_thread: int, groups_per_cu: int):
    _check(lib().lbm_batch_set_launch(b, nodes_per_thread, groups_per_cu), "lbm_batch_set_launch")


def lbm_batch_set_fusion(b: int, strip_rows: int):
    _check(lib().lbm_batch_set_fusion(b, strip_rows), "lbm_batch_set_fusion")


def lbm_batch_set_fusion_depth(b: int, steps: int):
    _check(lib().lbm_batch_set_fusion_depth(b, steps), "lbm_batch_set_fusion_depth")


def lbm_batch_get_fusion_depth(b: int) -> int:
    v = _i(0)
    _check(lib().lbm_batch_get_fusion_depth(b, ctypes.byref(v)), "lbm_batch_get_fusion_depth")
    return v.value


def lbm_batch_get_fusion(b: int) -> int:
    v = ctypes.c_int(0)
    _check(lib().lbm_batch_get_fusion(b, ctypes.byref(v)), "lbm_batch_get_fusion")
    return v.value


def lbm_batch_autotune(b: int, trials: int):
    npt, gpc, us = _i(), _i(), _d()
    _check(lib().lbm_batch_autotune(b, trials, ctypes.byref(npt), ctypes.byref(gpc), ctypes.byref(us)),
           "lbm_batch_autotune")
    return npt.value, gpc.value, us.value


def lbm_batch_residency(b: int, shape: int):
    """(groups per CU from the kernel's resources, runtime occupancy figure, confirmed figure,
    residency probes that had to lower a figure)."""
    vals = [_i() for _ in range(4)]
    _check(lib().lbm_batch_residency(b, shape, *(ctypes.byref(v) for v in vals)), "lbm_batch_residency")
    return tuple(v.value for v in vals)


def lbm_batch_destroy(b: int):
    lib().lbm_batch_destroy(b)


def lbm_state_bytes(ctx: int) -> int:
    return int(lib().lbm_state_bytes(ctx))


def lbm_adjoint_bytes(ctx: int) -> int:
    return int(lib().lbm_adjoint_bytes(ctx))


def lbm_save_state(ctx: int, dst: int):
    _check(lib().lbm_save_state(ctx, dst), "lbm_save_state")


def lbm_load_state(ctx: int, src: int, step: int):
    _check(lib().lbm_load_state(ctx, src, step), "lbm_load_state")


def lbm_step_raw(ctx: int, model: int, omega, src: int, dst: int, step: int):
    _check(lib().lbm_step_raw(ctx, model, _omega(omega), src, dst, step), "lbm_step_raw")


def _ptrs(seq):
    return (_vp * max(1, len(seq)))(*[int(p) for p in seq])


def lbm_step_raw_many(ctx: int, model: int, omega, src, dst, step0: int):
    _check(lib().lbm_step_raw_many(ctx, model, _omega(omega), _ptrs(src), _ptrs(dst), len(src), step0),
           "lbm_step_raw_many")


def lbm_step2_raw_many(ctx: int, model: int, omega, src, mid, dst, step0: int):
    """Pairs of raw steps src[k] -> dst[k]; mid[k] (0 / None = not kept) receives the state between."""
    mids = None if mid is None else _ptrs([m or 0 for m in mid])
    _check(lib().lbm_step2_raw_many(ctx, model, _omega(omega), _ptrs(src), mids, _ptrs(dst), len(src), step0),
           "lbm_step2_raw_many")


def lbm_step3_raw_many(ctx: int, model: int, omega, src, dst, step0: int):
    """Triples of raw steps src[k] -> dst[k] (the two states between are not written)."""
    _check(lib().lbm_step3_raw_many(ctx, model, _omega(omega), _ptrs(src), _ptrs(dst), len(src), step0),
           "lbm_step3_raw_many")


def lbm_adjoint_many(ctx: int, model: int, omega, states, lam, domega: int | None):
    _check(lib().lbm_adjoint_many(ctx, model, _omega(omega), _ptrs(states), len(states), _ptrs(lam),
                                  domega or None), "lbm_adjoint_many")


def lbm_adjoint_flush(ctx: int, domega: int):
    _check(lib().lbm_adjoint_flush(ctx, domega), "lbm_adjoint_flush")


def lbm_set_adjoint_depth(ctx: int, steps: int):
    _check(lib().lbm_set_adjoint_depth(ctx, steps), "lbm_set_adjoint_depth")


def lbm_get_adjoint_depth(ctx: int) -> int:
    steps = ctypes.c_int(0)
    _check(lib().lbm_get_adjoint_depth(ctx, ctypes.byref(steps)), "lbm_get_adjoint_depth")
    return steps.value


def lbm_adjoint_seed_velocity_l2(ctx: int, ux_t: int, uy_t: int, lam: int) -> float:
    loss = _d()
    _check(lib().lbm_adjoint_seed_velocity_l2(ctx, ux_t, uy_t, lam, ctypes.byref(loss)),
           "lbm_adjoint_seed_velocity_l2")
    return loss.value


def lbm_adjoint_step(ctx: int, model: int, omega, state: int | None, lam_next: int, lam: int, domega: int):
    _check(lib().lbm_adjoint_step(ctx, model, _omega(omega), state, lam_next, lam, domega),
           "lbm_adjoint_step")


def lbm_eq_vjp(ctx: int, rho0: int, ux0: int, uy0: int, lam0: int, dux: int, duy: int):
    _check(lib().lbm_eq_vjp(ctx, rho0, ux0, uy0, lam0, dux, duy), "lbm_eq_vjp")


def lbm_last_error() -> str:
    return lib().lbm_last_error().decode(errors="replace")


def make_lsa_points(points) -> ctypes.Array:
    """Array of LsaPoint from dicts with model (code), eq_order, omega, ux, uy."""
    arr = (LsaPoint * len(points))()
    for a, d in zip(arr, points):
        a.model, a.eq_order = int(d["model"]), int(d["eq_order"])
        for k in range(5):
            a.omega[k] = float(d["omega"][k])
        a.ux, a.uy = float(d["ux"]), float(d["uy"])
    return arr


def lbm_lsa_jacobian(points: ctypes.Array, J: int, stream=None):
    _check(lib().lbm_lsa_jacobian(ctypes.cast(points, _vp), len(points), J, stream), "lbm_lsa_jacobian")


def lbm_lsa_eigenvalues(points: ctypes.Array, kx: int, ky: int, nk: int, lam: int, stream=None):
    _check(lib().lbm_lsa_eigenvalues(ctypes.cast(points, _vp), kx, ky, nk, lam, stream), "lbm_lsa_eigenvalues")


def lbm_lsa_radius(points: ctypes.Array, kx: int, ky: int, nk: int, radius: int, stream=None):
    _check(lib().lbm_lsa_radius(ctypes.cast(points, _vp), len(points), kx, ky, nk, radius, stream), "lbm_lsa_radius")


def lbm_lsa_dvbe_growth(points: ctypes.Array, tau: float, kx: int, ky: int, nk: int, growth: int, stream=None):
    _check(lib().lbm_lsa_dvbe_growth(ctypes.cast(points, _vp), len(points), float(tau), kx, ky, nk, growth, stream),
           "lbm_lsa_dvbe_growth")
