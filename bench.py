"""Throughput of the fused D2Q9 stream-and-collide step on one MI355X.

Workload: 4096 x 4096 periodic double shear layer (Ma = 0.1, rho0 = 1, Re = 3e4 so
nu = U L / Re), populations stored as shifted FP32 deviations, REG relaxation rates.  One
bench step advances the grid by one time step with each of the eight collision models (eight
independent grids, one launch each), so `value` is the aggregate MLUPS over the models and
`per_model` gives each model's own rate.  Inputs are resident in HBM before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec f32|f64|f16] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E spec


def bytes_per_cell(prec: str) -> int:
    return 18 * {"f64": 8, "f32": 4, "f16": 2}[prec]


def cpu_baseline(models, budget_s: float = 16.0):
    """The oracle (single-threaded FP64) on a bounded sample: 256 x 256 double shear layer,
    each model run for whole steps until its share of the time budget is used."""
    import oracle
    from paper_2002_05265_amd import inputs

    n = 256
    rho, ux, uy = inputs.dsl_fields(n, n, 0.1)
    omega = inputs.rates(inputs.dsl_nu(n), "REG")
    f0 = oracle.init_eq(4, rho, ux, uy)
    updates, elapsed, steps_done = 0, 0.0, {}
    for name in models:
        t0 = time.perf_counter()
        f, k = f0, 0
        while True:
            f = oracle.step(f, oracle.MODELS[name], 4, omega, 1)
            k += 1
            if time.perf_counter() - t0 > budget_s / len(models):
                break
        elapsed += time.perf_counter() - t0
        updates += n * n * k
        steps_done[name] = k
    return {"value": updates / elapsed / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{n}x{n} double shear layer, FP64, steps per model {steps_done}, "
                      f"{elapsed:.1f} s total"}


def time_models(prec: str, n: int, models, steps: int, warmup: int, omega, fields):
    """Per-model timing of `steps` launches on an n x n grid (HIP events on the launch stream)."""
    import torch

    from paper_2002_05265_amd.sim import Sim

    out = {}
    for m in models:
        s = Sim(*fields, prec=prec, eq_order=4, device="cuda:0")
        s.step(m, omega, warmup)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        s.step(m, omega, steps)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / steps
        mlups = n * n / us
        gbs = mlups * 1e6 * bytes_per_cell(prec) / 1e9
        out[m] = {"mlups": round(mlups, 1), "us_per_step": round(us, 2), "hbm_gbs": round(gbs, 1),
                  "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "blowup": s.status()[1]}
        s.close()
        del s
        torch.cuda.empty_cache()
    return out


def batched_sweep(steps: int, plain_f64_mlups: float, n_inst: int = 512):
    """Random stability sweep: n_inst instances (side in {64..512}, Ma in [0, 0.6], log10 nu in
    [-7, -2], model uniform over the eight, one Fourier-mode perturbation of amplitude 1e-3),
    FP64, advanced by one persistent launch.  Throughput counts the nodes actually updated
    (an instance stops after the step at which it blew up)."""
    import torch

    from paper_2002_05265_amd import inputs
    from paper_2002_05265_amd.batch import Batch
    from paper_2002_05265_amd.sim import Sim

    insts = inputs.sweep_instances(n_inst)
    for k, d in enumerate(insts):
        d["omega"] = inputs.rates(d["nu"], "SRT" if k % 2 == 0 else "REG")
        d["eq_order"] = 4
    fields = [inputs.sweep_fields(d) for d in insts]
    b = Batch(insts, fields, prec="f64", device="cuda:0")
    tuned = b.autotune(3)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    b.run(steps)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    _, blow = b.status()
    b.close()
    del b
    torch.cuda.empty_cache()
    updates = sum(d["nx"] * d["ny"] * (steps if bl < 0 else min(bl + 1, steps)) for d, bl in zip(insts, blow))
    mlups = updates / sec / 1e6
    # the same instances through the plain kernel, one launch per instance and step
    ps = 50
    sims = [Sim(*f, prec="f64", eq_order=4, device="cuda:0") for f in fields]
    torch.cuda.synchronize()
    e0.record()
    for d, s in zip(insts, sims):
        s.step(d["model"], d["omega"], ps)
    e1.record()
    torch.cuda.synchronize()
    plain_sec = e0.elapsed_time(e1) * 1e-3
    plain_updates = sum(d["nx"] * d["ny"] * ps for d in insts)
    for s in sims:
        s.close()
    del sims
    torch.cuda.empty_cache()
    return {"instances": n_inst, "steps": steps, "seconds": round(sec, 3),
            "active_updates": updates, "mlups": round(mlups, 1),
            "vs_plain_f64_4096": round(mlups / plain_f64_mlups, 3),
            "plain_same_instances_mlups": round(plain_updates / plain_sec / 1e6, 1),
            "vs_plain_same_instances": round(mlups / (plain_updates / plain_sec / 1e6), 3),
            "blown_up": int(sum(1 for bl in blow if bl >= 0)),
            "blowup_steps_first10": blow[:10],
            "autotuned": {"nodes_per_thread": tuned[0], "groups_per_cu": tuned[1]},
            "precision": "f64"}


def adjoint_run(n: int = 512, steps: int = 2000, prec: str = "f32"):
    """Vortex-transport gradient: n x n CM convected vortex (Ma 0.2, nu 1e-5, REG rates),
    L = ||u_T - u_target||_2 after `steps`, gradients w.r.t. the initial velocity field and the
    rates by the discrete adjoint with sqrt(n) checkpoints.  Compared with the plain forward
    run of the same grid, precision and step count."""
    import torch

    from paper_2002_05265_amd import inputs
    from paper_2002_05265_amd.adjoint import _Run
    from paper_2002_05265_amd.sim import Sim

    mach = 0.2
    rho, ux, uy = inputs.vortex_fields(n, n, mach, beta=0.15, radius_frac=0.1)
    tx, ty = inputs.translated_vortex_velocity(n, n, mach, steps, beta=0.15, radius_frac=0.1)
    omega = inputs.rates(1e-5, "REG")
    uref = (mach * inputs.CS, 0.0)
    dev = torch.device("cuda:0")
    u0 = torch.tensor(np.stack([ux, uy]), device=dev)
    tgt = torch.tensor(np.stack([tx, ty]), device=dev)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    # plain forward
    sim = Sim(rho, ux, uy, prec=prec, eq_order=4, device=dev, ref_velocity=uref)
    sim.step("CM", omega, 20)
    torch.cuda.synchronize()
    e[0].record()
    sim.step("CM", omega, steps)
    e[1].record()
    torch.cuda.synchronize()
    plain_s = e[0].elapsed_time(e[1]) * 1e-3
    sim.close()
    run = _Run(u0, omega, torch.tensor(rho, device=dev), tgt, "CM", steps, prec, 4, "sqrt", 0, uref)
    torch.cuda.synchronize()
    e[0].record()
    loss = run.forward()
    e[1].record()
    e[2].record()
    du, dw = run.backward()
    e[3].record()
    torch.cuda.synchronize()
    fwd_s = e[0].elapsed_time(e[1]) * 1e-3
    bwd_s = e[2].elapsed_time(e[3]) * 1e-3
    stats = {"recomputed_steps": run.steps_run - steps, "peak_states": run.peak_states}
    run.close()
    total = fwd_s + bwd_s
    cells = n * n
    return {"workload": f"{n}x{n} CM convected vortex, Ma 0.2, nu 1e-5, REG, {prec} (mean-flow "
                        f"reference), {steps} steps, sqrt(n) checkpoints",
            "loss": loss, "grad_omega": [float(v) for v in dw.cpu()],
            "forward_s": round(fwd_s, 4), "backward_s": round(bwd_s, 4),
            "plain_forward_s": round(plain_s, 4),
            "mlups_forward_plus_backward": round(cells * steps / total / 1e6, 1),
            "plain_mlups": round(cells * steps / plain_s / 1e6, 1),
            "vs_plain": round(plain_s / total, 3),
            "expected_vs_plain_from_bytes": round(18 / (18 + 18 + 27), 3),
            "cache_resident": True, **stats}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--prec", default="f32", choices=["f32", "f64", "f16"])
    ap.add_argument("--models", default="BGK,RM,HM,CM,CHM,K,PR,RR")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64/FP16, batched and adjoint measurements")
    ap.add_argument("--batch-steps", type=int, default=20000)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the grid would shard as y-slabs with a one-row halo; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2002_05265_amd import inputs
    from paper_2002_05265_amd.sim import Sim

    torch.cuda.set_device(0)
    if args.copy_probe:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 1 << 30, "copy_probe_bytes_written": 1 << 30,
                          "launches": 5}), flush=True)
        return
    models = args.models.split(",")
    n = args.n
    mach = 0.1
    nu = inputs.dsl_nu(n, mach)
    omega = inputs.rates(nu, "REG")
    rho, ux, uy = inputs.dsl_fields(n, n, mach)
    sims = {m: Sim(rho, ux, uy, prec=args.prec, eq_order=4, device="cuda:0") for m in models}
    for m, s in sims.items():
        s.step(m, omega, args.warmup)
    torch.cuda.synchronize()

    ev = {m: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for m in models}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m, s in sims.items():
        ev[m][0].record()
        s.step(m, omega, args.steps)
        ev[m][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    cells = n * n
    per_model = {}
    for m in models:
        ms = ev[m][0].elapsed_time(ev[m][1])
        mlups = cells * args.steps / (ms * 1e-3) / 1e6
        gbs = mlups * 1e6 * bytes_per_cell(args.prec) / 1e9
        per_model[m] = {"mlups": round(mlups, 1), "us_per_step": round(ms * 1e3 / args.steps, 2),
                        "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    status = {m: s.status() for m, s in sims.items()}
    value = cells * args.steps * len(models) / wall / 1e6
    dominant = max(models, key=lambda m: per_model[m]["us_per_step"])
    dom_us = per_model[dominant]["us_per_step"]
    achieved = cells * bytes_per_cell(args.prec) / (dom_us * 1e-6) / 1e9
    line = {
        "metric": "MLUPS per collision model at 4096^2 FP32 + % HBM roofline; adjoint/batched vs plain",
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "f16": "f16-storage/f32"}[args.prec],
        "data": "synthetic: analytic double shear layer initial condition",
        "config": {"workload": f"D2Q9 periodic double shear layer {n}x{n}, Ma=0.1, Re=3e4, "
                               f"{'shifted ' if args.prec != 'f64' else ''}{args.prec} populations, "
                               f"REG rates, 8 collision models (one grid each)",
                   "nx": n, "ny": n, "models": models, "omega": [round(w, 6) for w in omega]},
        "roofline": {"bound": "hbm", "kernel": f"k_step<{dominant}>", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "per_model": per_model,
        "blowup": {m: st[1] for m, st in status.items()},
    }
    for s in sims.values():
        s.close()
    del sims
    torch.cuda.empty_cache()
    if not args.no_extras:
        fields = (rho, ux, uy)
        extra_steps = max(20, args.steps // 2)
        line["precisions"] = {p: time_models(p, n, models, extra_steps, 5, omega, fields) for p in ("f64", "f16")}
        f64_mlups = min(v["mlups"] for v in line["precisions"]["f64"].values())
        line["batched"] = batched_sweep(args.batch_steps, f64_mlups)
        line["adjoint"] = adjoint_run()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(models)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
