"""Numerical stability domains of the collision models (Section 5b-c), on the batched kernel.

Every point (collision model, relaxation preset, viscosity nu, Mach number Ma) is one run of the
convected vortex of Section 5a on a periodic L x L grid (beta = 0.5, R = L / 20, mean flow along
x), advanced for M convective times t_c = L / u0 (u0 = Ma cs).  A run is unstable if the domain
mean of |u|^2 rises above its initial value at any check up to M t_c (the quantity is expected to
decrease monotonically), or if the state blows up (a node with !(rho > 0)).  All runs of a map
are instances of one batch; |u|^2 is checked every `check_every` steps and at each run's own
last step, and a run leaves the batch once it is classified.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import inputs
from .batch import Batch


def vortex_instances(models, presets, nus, machs, L: int, M: float, eq_order: int = 4):
    """One instance description per (model, preset, nu, Ma), with its step budget M t_c."""
    out = []
    for model in models:
        for preset in presets:
            for nu in nus:
                for ma in machs:
                    out.append({"nx": L, "ny": L, "model": model, "preset": preset, "nu": float(nu),
                                "mach": float(ma), "eq_order": eq_order,
                                "omega": inputs.rates(float(nu), preset),
                                "budget": int(math.ceil(M * L / (ma * inputs.CS)))})
    return out


def check_schedule(budgets, check_every: int = 64):
    """Steps at which |u|^2 is checked: `check_every` steps after the previous check, or earlier
    when a run's budget comes first (every budget is a check)."""
    stops = np.unique(np.asarray(budgets, dtype=np.int64))
    out, step = [], 0
    while step < stops[-1]:
        step = min(step + check_every, int(stops[np.searchsorted(stops, step, side="right")]))
        out.append(step)
    return out


def vortex_field(d, beta: float = 0.5, radius_frac: float = 0.05):
    """Initial fields of a convected-vortex instance (Section 5a)."""
    return inputs.vortex_fields(d["nx"], d["ny"], d["mach"], beta=beta, radius_frac=radius_frac)


def dsl_field(d):
    """Initial fields of a double-shear-layer instance (Appendix C)."""
    return inputs.dsl_fields(d["nx"], d["ny"], d["mach"])


def dsl_instances(models_presets, Ls, machs, M: float, reynolds: float = 3.0e4):
    """Double shear layer runs (Appendix C) at Re = u0 L / nu, one per ((model, preset), L, Ma),
    each with its budget of M convective times t_c = L / u0."""
    out = []
    for model, preset in models_presets:
        for L in Ls:
            for ma in machs:
                nu = inputs.dsl_nu(L, ma, reynolds)
                out.append({"nx": L, "ny": L, "model": model, "preset": preset, "nu": float(nu), "mach": float(ma),
                            "eq_order": 4, "omega": inputs.rates(float(nu), preset),
                            "budget": int(math.ceil(M * L / (ma * inputs.CS)))})
    return out


def run_stability(instances, prec: str = "f64", check_every: int = 64, beta: float = 0.5,
                  radius_frac: float = 0.05, device="cuda:0", autotune: bool = True,
                  criterion: str = "u2", field=None, progress_s: float = 0.0):
    """Classify every instance; returns (first_bad_step per instance (-1 = stable), seconds of GPU
    time, node updates performed).  criterion "u2" is the |u|^2 test above; "blowup" counts only
    a loss of positivity within the budget.  field(d) gives an instance's initial (rho, ux, uy);
    the default is the convected vortex with beta and radius_frac.  progress_s > 0 prints the step
    and the number of live runs at most that often (host time)."""
    if field is None:
        fields = [vortex_field(d, beta, radius_frac) for d in instances]
    else:
        fields = [field(d) for d in instances]
    dev = torch.device(device)
    b = Batch(instances, fields, prec=prec, device=dev)
    try:
        if autotune:
            b.autotune(3)
        n = b.n
        budgets = np.array([d["budget"] for d in instances], dtype=np.int64)
        cells = torch.tensor([d["nx"] * d["ny"] for d in instances], dtype=torch.float64, device=dev)
        budget_d = torch.tensor(budgets, device=dev)
        u2_0 = b.mean_u2().clone()
        u2 = torch.empty_like(u2_0)
        first_bad = torch.full((n,), -1, dtype=torch.int64, device=dev)
        active = torch.ones(n, dtype=torch.int32, device=dev)
        updates = torch.zeros((), dtype=torch.float64, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step, k_chunk = 0, 0
        t_last = time.perf_counter()
        for nxt in check_schedule(budgets, check_every):
            k = nxt - step
            updates += (active.to(torch.float64) * cells).sum() * k
            b.run(k)
            step = nxt
            live = active.bool()
            if criterion == "u2":
                b.mean_u2(u2)
                bad = live & ~(u2 <= u2_0)       # rises above the start, or NaN
            else:
                bad = torch.zeros_like(live)
            first_bad = torch.where(bad & (first_bad < 0), torch.full_like(first_bad, step), first_bad)
            active = (live & ~bad & (budget_d > step)).to(torch.int32)
            b.set_active(active)
            k_chunk += 1
            if k_chunk % 16 == 0:
                live_n = int(active.sum())
                if live_n == 0:
                    break
                b.rebalance()  # retired runs leave the per-XCD work lists
                if progress_s > 0 and time.perf_counter() - t_last > progress_s:
                    t_last = time.perf_counter()
                    print(f"stability: step {step}, {live_n} of {n} runs live", flush=True)
        e1.record()
        _, blow = b.status()
        sec = e0.elapsed_time(e1) * 1e-3
        fb = first_bad.cpu().numpy()
        blow = np.asarray(blow)
        # a blow-up inside the budget that the |u|^2 checks did not see is unstable too
        missed = (fb < 0) & (blow >= 0) & (blow < budgets)
        fb[missed] = blow[missed]
        return fb, sec, float(updates)
    finally:
        b.close()


def max_stable_mach(instances, first_bad):
    """{(model, preset, nu): largest Ma of the grid below which every Ma is stable (0 if the
    smallest is unstable)}."""
    groups = {}
    for d, fb in zip(instances, first_bad):
        groups.setdefault((d["model"], d["preset"], d["nu"]), []).append((d["mach"], fb < 0))
    out = {}
    for key, pts in groups.items():
        best = 0.0
        for ma, stable in sorted(pts):
            if not stable:
                break
            best = ma
        out[key] = best
    return out
