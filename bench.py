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
ROOT = os.path.dirname(os.path.abspath(__file__))
PROFILE_DIR = os.path.join(ROOT, "profiles")
# the sources the plain step kernel is compiled from: a measured traffic figure is reported only
# while these are unchanged since the counters were taken
STEP_SOURCES = ("paper_2002_05265_amd/csrc/lbm_core.hip", "paper_2002_05265_amd/csrc/lbm_cell.hpp",
                "paper_2002_05265_amd/csrc/lbm_internal.hpp", "paper_2002_05265_amd/csrc/lbm_step2.hpp",
                "paper_2002_05265_amd/csrc/lbm_step3.hpp", "paper_2002_05265_amd/build.py")
MODEL_ORDER = ("BGK", "RM", "HM", "CM", "CHM", "K", "PR", "RR")
PREC_CODE = {"f64": 0, "f32": 1, "f16": 2}


def bytes_per_cell(prec: str) -> int:
    return 18 * {"f64": 8, "f32": 4, "f16": 2}[prec]


def step_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for rel in STEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(rel.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def step_kernel_keys(model: str, prec: str):
    """(label, name prefix in a kernel trace) of the three-step kernels (64-column and narrow
    strips), the two-step and the single-step kernel."""
    args = f"{MODEL_ORDER.index(model)}, {PREC_CODE[prec]}, "
    return [("k_step3", f"k_step3<{args}"), ("k_step3n", f"k_step3n<{args}"), ("k_step2", f"k_step2<{args}"),
            ("k_step", f"k_step<{args}")]


def repeated_windows(sims, models, omega, steps: int, k: int = 5):
    """Issue k more windows of `steps` steps per model, back to back on each model's grid (the
    grids keep advancing; the rate does not depend on the data), with a HIP event after each; read
    them with repeats_from after a synchronisation."""
    import torch

    evs = {}
    for m in models:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
        ev[0].record()
        for i in range(k):
            sims[m].step(m, omega, steps)
            ev[i + 1].record()
        evs[m] = ev
    return evs


def repeats_from(evs, cells: int, steps: int):
    """Median and relative spread of each model's repeated windows, next to the one timed window of
    the headline figure."""
    import statistics

    out = {}
    for m, ev in evs.items():
        rates = [cells * steps / (ev[i].elapsed_time(ev[i + 1]) * 1e-3) / 1e6 for i in range(len(ev) - 1)]
        med = statistics.median(rates)
        out[m] = {"median_mlups": round(med, 1), "spread": round((max(rates) - min(rates)) / med, 4)}
    return {"windows": len(next(iter(evs.values()))) - 1, "steps": steps, "per_model": out}


def fused_launch_windows(sims, models, omega, steps: int):
    """Issue max(4, steps / steps per launch) whole fused launches (no leftover launch of fewer
    steps) per model in one call each, between two HIP events; launch_us_from reads the average
    launch duration after a synchronisation."""
    import torch

    ev = {}
    for m in models:
        s = sims[m]
        spl = launch_steps(s, m)
        nl = max(4, steps // spl)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(m, omega, nl * spl)
        e1.record()
        ev[m] = (e0, e1, nl)
    return ev


def launch_us_from(ev):
    return {m: e0.elapsed_time(e1) * 1e3 / nl for m, (e0, e1, nl) in ev.items()}


def launch_steps(sim, model: str) -> int:
    """Steps one launch of `model` advances on `sim`: 3, 2 or 1."""
    ring = sim.fusion(model)[0]
    if not ring:
        return 1
    return 3 if sim.fusion_depth(model) == 3 and ring in (4, 8) else 2


def profile_path(prec: str, kind: str) -> str:
    return os.path.join(PROFILE_DIR, f"step_kernels_{prec}_dsl4096_{kind}.md")


def counter_record(model: str, prec: str):
    """The step kernel's record in the committed counter summary (HBM bytes, VALUBusy, flops per
    node update), or None when there is none for this kernel or its sources changed since the
    counters were taken."""
    path = profile_path(prec, "counters")
    try:
        with open(path) as fh:
            text = fh.read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("step_source_hash") != step_source_hash():
        return None
    return blob.get("per_launch", {}).get(model)


def measured_traffic(model: str, prec: str):
    """HBM bytes per launch of the step kernel from the committed counter summary, or None."""
    rec = counter_record(model, prec)
    return None if rec is None else rec["hbm_bytes"]


def measured_valu_busy(model: str, prec: str):
    """Fraction of the vector-ALU issue capacity the step kernel used (rocprofv3 VALUBusy) from the
    committed counter summary, or None."""
    rec = counter_record(model, prec)
    return None if rec is None or rec.get("valu_busy") is None else rec["valu_busy"]


# FP32 / FP64 vector peaks of MI355X (256 CUs at 2.4 GHz): 157.3 TFLOP/s counts packed FP32 FMAs
# (two per lane and cycle), 78.6 TFLOP/s one FMA per lane and cycle (FP64, or FP32 built without
# packed FP32, as this library is)
VECTOR_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
UNPACKED_PEAK_TFLOPS = 78.6
VALU_BOUND = 0.85  # VALUBusy from which a kernel counts as bound by vector-ALU issue


def limiter(rec, hbm_frac_measured):
    """What bounds a step kernel, from its counters: vector-ALU issue (VALUBusy >= 0.85), HBM
    (measured traffic >= 0.8 of the peak), else neither: the pass structure / latency."""
    if rec is None:
        return None
    if rec.get("valu_busy") is not None and rec["valu_busy"] >= VALU_BOUND:
        return "valu-issue"
    if hbm_frac_measured is not None and hbm_frac_measured >= 0.8:
        return "hbm"
    return "pass-structure/latency"


def roofline_block(model, prec, kname, cells, bpc, spl, launch_us, stream_launch_us, n):
    """Roofline entry of the dominant kernel.  The bound comes from its counters: vector-ALU issue
    gives "alu" with the algorithmic flops (the single-step kernel's flops per node update x nodes x
    steps per launch) over the launch time against the FP32 (FP64) vector peak; otherwise "hbm"
    with the algorithmic bytes per launch (each population read and written once) over the launch
    time against 8 TB/s.  Both views are reported either way, with the per-update HBM figure of the
    18 s bytes-per-node-and-step model (above 1 when a launch advances several steps per read)."""
    rec = counter_record(model, prec) if n == 4096 else None
    traffic = None if rec is None else rec["hbm_bytes"]
    valu_busy = None if rec is None else rec.get("valu_busy")
    fpu = None if rec is None else rec.get("flops_per_update")
    gbs = cells * bpc / (launch_us * 1e-6) / 1e9
    measured_frac = None if traffic is None else traffic / (launch_us * 1e-6) / 1e9 / HBM_PEAK_GBS
    hbm = {"achieved_gbs": round(gbs, 1), "frac_at_bytes_per_launch": round(gbs / HBM_PEAK_GBS, 4),
           "per_update_gbs": round(gbs * spl, 1), "frac_at_18s_bytes_per_update": round(gbs * spl / HBM_PEAK_GBS, 4),
           "measured_frac": None if measured_frac is None else round(measured_frac, 4),
           "stream_only_gbs": round(cells * bpc / (stream_launch_us * 1e-6) / 1e9, 1),
           "frac_of_stream_only": round(stream_launch_us / launch_us, 4)}
    alu = None
    if fpu is not None:
        tf = fpu * cells * spl / (launch_us * 1e-6) / 1e12
        peak = VECTOR_PEAK_TFLOPS[prec if prec == "f64" else "f32"]
        alu = {"achieved_tflops": round(tf, 2), "peak_tflops": peak, "frac": round(tf / peak, 4),
               "frac_of_unpacked_peak": round(tf / UNPACKED_PEAK_TFLOPS, 4),
               "flops_per_update": fpu, "executed_flops_per_update": rec.get("executed_flops_per_update")}
    lim = limiter(rec, measured_frac)
    common = {"kernel": f"{kname}<{model}>", "limiter": lim, "valu_busy": valu_busy, "traffic": traffic,
              "traffic_unit": "HBM bytes per launch (counters)", "algorithmic_bytes": cells * bpc,
              "launch_us": round(launch_us, 2), "steps_per_launch": spl, "hbm": hbm, "alu": alu}
    if lim == "valu-issue" and alu is not None:
        return {"bound": "alu", "achieved": alu["achieved_tflops"], "peak": alu["peak_tflops"], "unit": "TFLOP/s",
                "frac": alu["frac"], **common}
    return {"bound": "hbm", "achieved": hbm["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": hbm["frac_at_bytes_per_launch"], **common}


def _oracle_rate(job):
    """One model's oracle run (single-threaded FP64 C, in a spawned process): MLUPS on the n x n
    double shear layer (the bench workload's field and rates at that size), `steps` steps."""
    name, n, steps = job
    import oracle
    from paper_2002_05265_amd import inputs

    rho, ux, uy = inputs.dsl_fields(n, n, 0.1)
    omega = inputs.rates(inputs.dsl_nu(n), "REG")
    f0 = oracle.init_eq(4, rho, ux, uy)
    del rho, ux, uy
    t0 = time.perf_counter()
    f = oracle.step(f0, oracle.MODELS[name], 4, omega, steps)
    dt = time.perf_counter() - t0
    del f, f0
    return name, n, steps, n * n * steps / dt / 1e6, dt


def host_cpu():
    """(CPU model name from /proc/cpuinfo with its family / model / stepping numbers, clock and
    cache size, which identify the generation where a virtual machine shows only a generic
    name; logical CPUs of the host; CPUs this process may use)."""
    cpu = "unknown"
    try:
        fields = {}
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if not ln.strip():
                    break  # the first processor's block
                k, _, v = ln.partition(":")
                fields[k.strip()] = v.strip()
        cpu = fields.get("model name", cpu)
        extra = [f"{k} {fields[k]}" for k in ("vendor_id", "cpu family", "model", "stepping", "cpu MHz",
                                              "cache size") if k in fields]
        if extra:
            cpu += " (" + ", ".join(extra) + ")"
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return cpu, os.cpu_count(), usable


def cpu_baseline(models, sizes=((1024, 100), (4096, 3)), procs: int = 8):
    """The oracle (single-threaded FP64 C) timed per model on the bench workload at two sizes:
    the double shear layer at 1024^2 for 100 steps and at the bench's 4096^2 for 3 steps.  Every
    run uses one core; the runs go to `procs` spawned processes at a time (each its own core), so
    the per-model rates are one-core rates.  `value` is the one-core rate of a bench step (one
    step of every model) at 4096^2: total updates over total one-core seconds."""
    import multiprocessing as mp

    cpu, ncpu, usable = host_cpu()
    jobs = [(m, n, st) for n, st in sizes for m in models]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(max(1, min(procs, usable or 1, len(jobs)))) as pool:
        res = pool.map(_oracle_rate, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    per_model = {m: {} for m in models}
    for name, n, st, mlups, dt in res:
        per_model[name][f"{n}x{n}x{st}"] = round(mlups, 3)
    big_n, big_st = sizes[-1]
    big = [(dt, n * n * st) for _, n, st, _, dt in res if n == big_n]
    value = sum(u for _, u in big) / sum(dt for dt, _ in big) / 1e6
    return {"value": round(value, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "host_cpu": cpu, "host_nproc": ncpu, "usable_cpus": usable, "per_model": per_model,
            "sample": (f"every model on the double shear layer at "
                       + " and ".join(f"{n}x{n} for {st} steps" for n, st in sizes)
                       + f" (FP64, one thread per run; {min(procs, usable or 1, len(jobs))} runs at a time "
                       f"in separate processes, {wall:.0f} s wall); value: one core's rate over one step of "
                       f"each model at {big_n}x{big_n}")}


def single_step_rates(sims, models, omega, cells, bpc, steps):
    """The same grids with one step per launch (fused launches switched off), for comparison;
    each sim's own setting is restored afterwards."""
    import torch

    out = {}
    for m in models:
        s = sims[m]
        ring, strip = s.fusion(m)
        s.set_fusion(m, 0)
        s.step(m, omega, 2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(m, omega, steps)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / steps
        s.set_fusion(m, ring, strip)
        out[m] = {"mlups": round(cells / us, 1), "hbm_gbs": round(cells * bpc / us / 1e3, 1)}
    return out


def cache_resident_rates(models, sizes=(1024, 512), precs=("f32", "f64"), steps: int = 200):
    """MLUPS on grids whose two copies fit the 256 MB last-level cache (the double shear layer at
    1024^2 and 512^2, the bench's default launch settings): labelled cache-resident, not compared
    with the HBM roofline."""
    from paper_2002_05265_amd import inputs

    out = {}
    for n in sizes:
        fields = inputs.dsl_fields(n, n, 0.1)
        omega = inputs.rates(inputs.dsl_nu(n), "REG")
        for prec in precs:
            r = time_models(prec, n, models, steps, 10, omega, fields)
            out[f"{prec}-{n}"] = {m: v["mlups"] for m, v in r.items()}
    return {"cache_resident": True, "steps": steps, "mlups": out}


def note(msg: str):
    """A progress line on stderr (the JSON result is the only line on stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


_SETTLE = {}


def settle_clocks(seconds: float = 0.3, prec: str = "f32", n: int = 4096):
    """Run the step kernels of the models on a scratch grid (not one of the timed grids) for
    `seconds` before the warm-up steps.  After an idle stretch (host-side set-up) MI355X runs the
    compute-heavy step kernels ~15% slower for some 10 ms once they resume, a power transient
    that memory copies do not condition away (measured), and which would fall into short timed
    windows."""
    import torch

    from paper_2002_05265_amd import inputs
    from paper_2002_05265_amd.sim import Sim

    key = (prec, n)
    if key not in _SETTLE:
        _SETTLE.clear()
        torch.cuda.empty_cache()
        _SETTLE[key] = Sim(*inputs.dsl_fields(n, n, 0.1), prec=prec, eq_order=4, device="cuda:0")
    s = _SETTLE[key]
    omega = inputs.rates(inputs.dsl_nu(n, 0.1), "REG")
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for m in MODEL_ORDER:
            s.step(m, omega, 3)
        torch.cuda.synchronize()


def release_settle():
    for s in _SETTLE.values():
        s.close()
    _SETTLE.clear()


def time_models(prec: str, n: int, models, steps: int, warmup: int, omega, fields):
    """Per-model timing of `steps` launches on an n x n grid (HIP events on the launch stream)."""
    import torch

    from paper_2002_05265_amd.sim import Sim

    out = {}
    for m in models:
        s = Sim(*fields, prec=prec, eq_order=4, device="cuda:0")
        settle_clocks(0.1, prec if prec != "f16" else "f32", min(n, 4096))
        s.step(m, omega, warmup)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        s.step(m, omega, steps)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / steps
        spl = launch_steps(s, m)
        mlups = n * n / us
        gbs = mlups * 1e6 * bytes_per_cell(prec) / spl / 1e9
        out[m] = {"mlups": round(mlups, 1), "us_per_step": round(us, 2), "steps_per_launch": spl,
                  "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "blowup": s.status()[1]}
        s.close()
        del s
        torch.cuda.empty_cache()
    return out


def batched_sweep(steps: int, plain_f64_mlups: float, n_inst: int = 512):
    """Random stability sweep: n_inst instances (side in {64..512}, Ma in [0, 0.6], log10 nu in
    [-7, -2], model uniform over the eight, one Fourier-mode perturbation of amplitude 1e-3),
    FP64, advanced by the persistent kernel (launch shape and one or two steps per pass
    autotuned) in pieces of 500 steps with the live instances re-dealt over the XCDs in between.  Throughput counts the nodes actually updated (an
    instance stops after the step at which it blew up)."""
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
    fused_rows = b.fusion()  # 0: one step per pass won the autotuning
    per_pass = b.fusion_depth() if fused_rows else 1
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    b.run(steps, rebalance_every=500)  # blown-up instances leave the per-XCD work lists
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
            "autotuned": {"nodes_per_thread": tuned[0], "groups_per_cu": tuned[1],
                          "steps_per_pass": per_pass, "strip_rows": fused_rows},
            "rebalance_every": 500, "precision": "f64"}


def stability_map(L: int = 32, M: float = 50.0, check_every: int = 64, progress_s: float = 0.0):
    """Numerical stability domains of the convected vortex (beta 0.5, R = L/20), every model under
    SRT and REG, nu in {1e-6 .. 1e-2}, Ma in {0.05 .. 0.8}, M convective times each, all runs in
    one batch (FP64).  Reports the largest stable Ma per model, preset and nu."""
    from paper_2002_05265_amd import inputs
    from paper_2002_05265_amd import stability as S

    nus = [1e-6, 1e-5, 1e-4, 1e-3, 1e-2]
    machs = [round(0.05 * k, 2) for k in range(1, 17)]
    insts = S.vortex_instances(list(inputs.MODEL_NAMES), ["SRT", "REG"], nus, machs, L=L, M=M)
    fb, sec, upd = S.run_stability(insts, check_every=check_every, progress_s=progress_s)
    best = S.max_stable_mach(insts, fb)
    table = {f"{m}-{p}": [best[(m, p, nu)] for nu in nus] for m in inputs.MODEL_NAMES for p in ("SRT", "REG")}
    return {"workload": f"convected vortex L={L}, M={M:g} t_c, {len(insts)} runs (8 models x SRT/REG x "
                        f"{len(nus)} nu x {len(machs)} Ma), FP64, |u|^2 criterion checked every "
                        f"{check_every} steps",
            "seconds": round(sec, 3), "node_updates": upd, "mlups": round(upd / sec / 1e6, 1),
            "nu": nus, "max_stable_mach": table}


def dsl_study():
    """Double shear layer (Re = 3e4): PR at Ma 0.12 on L = 128, 256, 512 (time of the instability,
    in t_c), and the largest stable Ma over 3 t_c of PR and RR on L = 128, 256."""
    from paper_2002_05265_amd import inputs
    from paper_2002_05265_amd import stability as S

    inst = S.dsl_instances([("PR", "REG")], [128, 256, 512], [0.12], M=3)
    fb, sec1, upd1 = S.run_stability(inst, field=S.dsl_field)
    times = {d["nx"]: (round(float(f) / (d["nx"] / (0.12 * inputs.CS)), 3) if f >= 0 else None)
             for d, f in zip(inst, fb)}
    machs = [round(0.02 * k, 2) for k in range(2, 36)]
    inst = S.dsl_instances([("PR", "REG"), ("RR", "SRT")], [128, 256], machs, M=3)
    fb, sec2, upd2 = S.run_stability(inst, field=S.dsl_field)
    pts = {}
    for d, f in zip(inst, fb):
        pts.setdefault(f"{d['model']}-L{d['nx']}", []).append((d["mach"], f))
    best = {}
    for key, v in pts.items():
        best[key] = 0.0
        for ma, f in sorted(v):
            if f >= 0:
                break
            best[key] = ma
    return {"workload": "double shear layer, Re 3e4, |u|^2 criterion, FP64",
            "pr_ma012_unstable_at_tc": times, "max_stable_mach_3tc": best,
            "seconds": round(sec1 + sec2, 3), "mlups": round((upd1 + upd2) / (sec1 + sec2) / 1e6, 1)}


def transport_study():
    """Convected vortex at Ma 0.5, nu 1e-4 over 50 t_c (SRT-RR, REG-CHM, REG-K; L = 256, 512):
    vorticity error against the initial field."""
    from paper_2002_05265_amd import accuracy as A

    res, tim = A.transport_accuracy([("RR", "SRT"), ("CHM", "REG"), ("K", "REG")], [256, 512])
    sec = sum(t for t, _ in tim.values())
    upd = sum(u for _, u in tim.values())
    return {"workload": "convected vortex Ma 0.5, nu 1e-4, 50 t_c, FP64",
            "metrics": {f"{m}-{p}-L{L}": {"l2": round(v["l2"], 6), "peak": round(v["peak"], 6),
                                            "shift": [round(x, 3) for x in v["shift"]]}
                        for (m, p, L), v in res.items()},
            "seconds": round(sec, 3), "mlups": round(upd / sec / 1e6, 1)}


def lsa_domain(n: int = 128):
    """Linear stability domain (Section 4c): every model under SRT and REG, nu in 1e-6 .. 1e-1,
    Ma in 0 .. 0.9, five flow directions in [0, pi/4], n x n wave numbers; largest stable Ma."""
    import math

    from paper_2002_05265_amd import inputs, lsa

    mp = [(m, p) for m in inputs.MODEL_NAMES for p in ("SRT", "REG")]
    nus = [1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1]
    machs = [round(0.025 * k, 3) for k in range(0, 37)]
    phis = list(np.linspace(0.0, math.pi / 4, 5))
    table, _, sec = lsa.stability_domain(mp, nus, machs, phis, n=n)
    mats = len(mp) * len(nus) * len(machs) * len(phis) * n * n
    # the BGK discrete-velocity Boltzmann equation (Section 3c): largest stable Ma on a 0.005 grid,
    # against sqrt(3) - 1 = 0.732
    dm = [round(0.005 * k, 3) for k in range(1, 200)]
    dvbe = {f"N{N}-phi{phi:.3f}": lsa.dvbe_critical_mach(N, phi, dm)
            for N, phi in ((2, 0.0), (2, math.pi / 8), (2, math.pi / 4), (4, 0.0), (4, math.pi / 4))}
    return {"workload": f"9x9 complex eigenproblems, {len(mp) * len(nus) * len(machs) * len(phis)} flows x {n}^2 "
                        "wave numbers, FP64", "seconds": round(sec, 3), "matrices_per_s": round(mats / sec, 1),
            "nu": nus, "max_stable_mach": {f"{m}-{p}": [table[(m, p, nu)] for nu in nus] for m, p in mp},
            "dvbe_max_stable_mach": dvbe}


def precision_errors(n: int = 4096, steps: int = 5000, models=("CM", "K")):
    """Shifted FP32 and FP16 storage against FP64 on the double shear layer: relative L2 error
    of the velocity field after `steps` steps (same initial fields, rates and model)."""
    import torch

    from paper_2002_05265_amd import inputs
    from paper_2002_05265_amd.sim import Sim

    mach = 0.1
    omega = inputs.rates(inputs.dsl_nu(n, mach), "REG")
    rho, ux, uy = inputs.dsl_fields(n, n, mach)
    out = {}
    for m in models:
        u = {}
        for p in ("f64", "f32", "f16"):
            s = Sim(rho, ux, uy, prec=p, eq_order=4, device="cuda:0")
            s.step(m, omega, steps)
            _, vx, vy, _ = s.moments()
            u[p] = torch.stack([vx, vy])
            s.close()
            del s
        norm = float(torch.linalg.vector_norm(u["f64"]))
        out[m] = {p: float(torch.linalg.vector_norm(u[p] - u["f64"])) / norm for p in ("f32", "f16")}
        del u
        torch.cuda.empty_cache()
    return {"workload": f"double shear layer {n}x{n}, Ma 0.1, Re 3e4, REG, {steps} steps",
            "l2_velocity_error_vs_f64": out}


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
    spl = launch_steps(sim, "CM")
    sim.close()
    # bytes per node the plain run's launches read and write: each population once per launch
    s_bytes = {"f64": 8, "f32": 4, "f16": 2}[prec]
    plain_node_bytes = 18 * s_bytes * (steps // spl + (1 if steps % spl else 0))
    rho_d = torch.tensor(rho, device=dev)
    # untimed warm-up sweep: first use of every kernel (and of torch's fill kernels) loads code
    # objects, a one-time host cost
    warm = _Run(u0, omega, rho_d, tgt, "CM", 16, prec, 4, "sqrt", 0, uref)
    warm.forward()
    warm.backward()
    warm.close()
    run = _Run(u0, omega, rho_d, tgt, "CM", steps, prec, 4, "sqrt", 0, uref)
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
    stats = {"recomputed_steps": run.steps_run - steps, "peak_states": run.peak_states,
             "plain_steps_per_launch": spl, "plain_bytes_per_node": plain_node_bytes,
             "adjoint_bytes_per_node": run.node_bytes}
    expected = plain_node_bytes / run.node_bytes
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
            "expected_vs_plain_from_bytes": round(expected, 3),
            "cache_resident": True, **stats}


def adjoint_step_rate(n: int, models, rho, ux, uy, omega, prec: str = "f32", steps: int = 20):
    """Throughput of the reverse steps alone at the bench grid.  One step per launch: a node of
    lambda_n = J_C^T S^T lambda_{n+1} reads 9 stored populations, gathers 9 adjoint values and
    writes 9 (27 values, 9 s + 18 a bytes).  Two per launch (three adjoint buffers in rotation):
    per node and pair, f_n, f_{n-1} and lambda_{n+1} read and lambda_{n-1} written (18 s + 18 a
    bytes, 9 s + 9 a per step).  Both against the same HBM peak as the forward step."""
    import torch

    from paper_2002_05265_amd import binding as B
    from paper_2002_05265_amd import inputs
    from paper_2002_05265_amd.sim import Sim

    sb, ab = (8, 8) if prec == "f64" else (4, 4)
    dev = torch.device("cuda:0")
    sim = Sim(rho, ux, uy, prec=prec, eq_order=4, device=dev)
    sim.step("CM", omega, 3)
    st = [torch.empty(B.lbm_state_bytes(sim.ctx), dtype=torch.uint8, device=dev) for _ in range(2)]
    B.lbm_save_state(sim.ctx, st[0].data_ptr())
    sim.step("CM", omega, 1)
    B.lbm_save_state(sim.ctx, st[1].data_ptr())
    lam = [torch.zeros(B.lbm_adjoint_bytes(sim.ctx), dtype=torch.uint8, device=dev) for _ in range(3)]
    states = [st[k % 2].data_ptr() for k in range(steps)]
    dw = torch.zeros(5, dtype=torch.float64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for depth, nbuf, key, bpn in ((1, 2, "one_step_per_launch", 9 * sb + 18 * ab),
                                  (2, 3, "two_steps_per_launch", 9 * sb + 9 * ab)):
        B.lbm_set_adjoint_depth(sim.ctx, depth)
        ptrs = [lam[k % nbuf].data_ptr() for k in range(steps + 1)]
        res = {}
        for m in models:
            code = inputs.MODEL_CODES[m]
            B.lbm_adjoint_many(sim.ctx, code, omega, states[:2], ptrs[:3], dw.data_ptr())
            torch.cuda.synchronize()
            e0.record()
            B.lbm_adjoint_many(sim.ctx, code, omega, states, ptrs, dw.data_ptr())
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / steps
            gbs = n * n * bpn / us / 1e3
            res[m] = {"us_per_step": round(us, 1), "mlups": round(n * n / us, 1), "gbs": round(gbs, 1),
                      "frac": round(gbs / HBM_PEAK_GBS, 4)}
        out[key] = {"bytes_per_node_and_step": bpn, "models": res}
    sim.close()
    return {"workload": f"reverse steps alone, {n}x{n} double shear layer states, {prec}, {steps} steps",
            **out}


def _csv_rows(path):
    import csv

    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find_csv(d, suffix):
    for f in sorted(os.listdir(d)):
        if f.endswith(suffix):
            return os.path.join(d, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def _per_dispatch(rows, key, counter=None):
    """Mean counter value per dispatch of every kernel whose name contains key (only rows of
    `counter` when given: a run that collects several counters has one row per counter)."""
    vals = [float(r["Counter_Value"]) for r in rows
            if key in r["Kernel_Name"] and (counter is None or r.get("Counter_Name") == counter)]
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


def flop_counters(prec: str):
    """The VALU instruction counters whose sum gives the floating-point operations of the
    arithmetic precision (FP32 for the shifted storages, FP64 otherwise); FMA counts twice."""
    t = "F64" if prec == "f64" else "F32"
    return [f"SQ_INSTS_VALU_ADD_{t}", f"SQ_INSTS_VALU_MUL_{t}", f"SQ_INSTS_VALU_FMA_{t}", f"SQ_INSTS_VALU_TRANS_{t}"]


def _flops_per_dispatch(rows, key, prec):
    """Floating-point operations per dispatch: 64 lanes x (add + mul + trans + 2 fma) wave instructions."""
    add, mul, fma, trans = (_per_dispatch(rows, key, c)[0] for c in flop_counters(prec))
    if None in (add, mul, fma, trans):
        return None
    return 64.0 * (add + mul + trans + 2.0 * fma)


def profile_summary(out_root: str, prec: str, n: int, commands: dict):
    """Write the kernel-trace and HBM-counter summaries of the bench workload under profiles/.

    out_root holds the rocprofv3 output directories rp_trace, rp_fetch, rp_write,
    rp_copy_fetch and rp_copy_write (csv format) written by the commands in `commands`."""
    os.makedirs(PROFILE_DIR, exist_ok=True)
    stats = _csv_rows(_find_csv(os.path.join(out_root, "rp_trace"), "kernel_stats.csv"))
    cells = n * n
    alg = cells * bytes_per_cell(prec)
    lines = [f"# k_step3 / k_step2 / k_step ({prec}, {n}x{n} double shear layer): kernel trace", "",
             "Command (from the repository root, with `cd /tmp && export TMPDIR=/tmp` semantics for",
             "the profiler's scratch files):", "", "```", commands["trace"], "```", "",
             f"Algorithmic bytes per launch: {n}*{n} nodes * 18 * {bytes_per_cell(prec) // 18} B = {alg} B "
             "(every population read and written once; k_step3 and k_step3n advance three steps per "
             "launch, k_step2 two, k_step one).",
             "", "| kernel | calls | average us | min us | max us | GB/s at algorithmic bytes |",
             "|---|---|---|---|---|---|"]
    for r in stats:
        name = r["Name"]
        short = name.replace("(anonymous namespace)::", "").replace("void ", "", 1).split("(")[0][:70]
        avg = float(r["AverageNs"]) * 1e-3
        gbs = ""
        for m in MODEL_ORDER:
            for label, key in step_kernel_keys(m, prec):
                if key in name:
                    gbs = f"{alg / (avg * 1e-6) / 1e9:.1f}"
                    short = f"{label}<{m}, {prec}>"
        lines.append(f"| {short} | {r['Calls']} | {avg:.2f} | {float(r['MinNs']) * 1e-3:.2f} | "
                     f"{float(r['MaxNs']) * 1e-3:.2f} | {gbs} |")
    with open(profile_path(prec, "trace"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    fetch = _csv_rows(_find_csv(os.path.join(out_root, "rp_fetch"), "counter_collection.csv"))
    write = _csv_rows(_find_csv(os.path.join(out_root, "rp_write"), "counter_collection.csv"))
    cfetch = _csv_rows(_find_csv(os.path.join(out_root, "rp_copy_fetch"), "counter_collection.csv"))
    cwrite = _csv_rows(_find_csv(os.path.join(out_root, "rp_copy_write"), "counter_collection.csv"))
    copy_key = "copyBuffer"  # the runtime's device-to-device copy kernel behind the 1 GiB copy
    valu_dir = os.path.join(out_root, "rp_valu")
    valu = _csv_rows(_find_csv(valu_dir, "counter_collection.csv")) if os.path.isdir(valu_dir) else []
    flops_dir = os.path.join(out_root, "rp_flops")
    flops = _csv_rows(_find_csv(flops_dir, "counter_collection.csv")) if os.path.isdir(flops_dir) else []
    cf, _ = _per_dispatch(cfetch, copy_key)
    cw, _ = _per_dispatch(cwrite, copy_key)
    gib_kib = (1 << 30) / 1024
    fscale, wscale = gib_kib / cf, gib_kib / cw
    per_launch = {}
    rows = ["| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) | / algorithmic | VALUBusy % "
            "| flops per node and step |",
            "|---|---|---|---|---|---|---|---|"]
    steps_of = {"k_step3": 3, "k_step3n": 3, "k_step2": 2, "k_step": 1}
    for m in MODEL_ORDER:
        # the first kernel of the model found (three-step, then two-step, then single-step) is the
        # one reported; the single-step kernel (no halo recomputation) gives the algorithmic flops
        # per node update
        single = _flops_per_dispatch(flops, step_kernel_keys(m, prec)[-1][1], prec)
        for label, key in step_kernel_keys(m, prec):
            f_kib, nf = _per_dispatch(fetch, key)
            w_kib, _ = _per_dispatch(write, key)
            if f_kib is None or w_kib is None:
                continue
            hbm = f_kib * 1024 * fscale + w_kib * 1024 * wscale
            vb, _ = _per_dispatch(valu, key)
            vtxt = "" if vb is None else f"{vb:.1f}"
            fl = _flops_per_dispatch(flops, key, prec)
            executed = None if fl is None else fl / (cells * steps_of[label])
            ftxt = "" if executed is None else f"{executed:.1f}"
            rows.append(f"| {label}<{m}, {prec}> | {nf} | {f_kib:.1f} | {w_kib:.1f} | {hbm:.4g} | {hbm / alg:.4f} | "
                        f"{vtxt} | {ftxt} |")
            per_launch.setdefault(m, {"kernel": label, "fetch_kib": round(f_kib, 1), "write_kib": round(w_kib, 1),
                                      "hbm_bytes": int(round(hbm)), "vs_algorithmic": round(hbm / alg, 4),
                                      "valu_busy": None if vb is None else round(vb / 100.0, 4),
                                      "flops_per_update": None if single is None else round(single / cells, 2),
                                      "executed_flops_per_update": None if executed is None else round(executed, 2)})
    blob = {"step_source_hash": step_source_hash(), "prec": prec, "n": n, "algorithmic_bytes": alg,
            "copy_probe_kib": {"fetch": round(cf, 1), "write": round(cw, 1), "true": gib_kib},
            "scale": {"fetch": round(fscale, 4), "write": round(wscale, 4)}, "per_launch": per_launch}
    text = [f"# k_step3 / k_step2 / k_step ({prec}, {n}x{n} double shear layer): HBM counters", "",
            "Commands (each counter in a run of its own):", "", "```", commands["fetch"], commands["write"],
            commands["copy_fetch"], commands["copy_write"], commands["valu"], commands["flops"], "```", "",
            "VALUBusy is rocprofv3's derived counter 100 * SQ_ACTIVE_INST_VALU / CUs / GRBM_GUI_ACTIVE: the "
            "share of the SIMDs' vector-ALU issue time in use (100 = every SIMD issues a VALU instruction "
            "every cycle it can).", "",
            "Flops per node and step: 64 lanes x (ADD + MUL + TRANS + 2 FMA) VALU instructions of the "
            "arithmetic's precision per dispatch (the SQ_INSTS_VALU_*_F32 or _F64 counters), over the nodes "
            "and steps the dispatch advances; the fused kernels' figure includes the halo recomputation. "
            "The single-step kernel's figure (`flops_per_update` below) is the algorithmic one.", "",
            "Calibration: a plain device copy of 1 GiB (torch, same box) reads "
            f"{cf:.1f} KiB of FETCH_SIZE and {cw:.1f} KiB of WRITE_SIZE per dispatch against "
            f"{gib_kib:.0f} KiB moved each way, so FETCH_SIZE is scaled by {fscale:.4f} and "
            f"WRITE_SIZE by {wscale:.4f}.", "", *rows, "",
            "Machine-readable (bench.py reports `roofline.traffic` from this block while the step "
            "kernel's sources hash to `step_source_hash`):", "", "```json", json.dumps(blob, indent=1), "```", ""]
    with open(profile_path(prec, "counters"), "w") as fh:
        fh.write("\n".join(text))
    print(json.dumps(blob), flush=True)


def extras_trace_summary(out_root: str, command: str):
    """Kernel-trace summary of a bench run with the extra workloads (every kernel of the batched,
    adjoint, stability and linear-analysis paths), written to profiles/."""
    d = os.path.join(out_root, "rp_trace_all")
    if not os.path.isdir(d):
        return
    stats = _csv_rows(_find_csv(d, "kernel_stats.csv"))
    lines = ["# All kernels of a bench run with the extra workloads: kernel trace", "",
             "Command (from the repository root):", "", "```", command, "```", "",
             "Under rocprofv3 this command ends with a segmentation fault (status 139) inside the C",
             "library's exit handlers, after the program has printed its JSON line and after the",
             "profiler's tool finalisation, with the result files complete; without the profiler it exits",
             "with status 0. By then the bench has closed every context and batch it made and the library",
             "holds nothing that is torn down at exit, so the fault is in the profiler's own exit path",
             "after cooperative launches. The batched launch shapes (one to three steps per pass) are",
             "autotuned inside the run, so a profiled run may pick other shapes than an unprofiled one.", "",
             "| kernel | calls | total ms | average us | share % |", "|---|---|---|---|---|"]
    for r in stats[:40]:
        name = r["Name"].replace("(anonymous namespace)::", "").replace("void ", "", 1).split("(")[0][:80]
        lines.append(f"| {name} | {r['Calls']} | {float(r['TotalDurationNs']) * 1e-6:.2f} | "
                     f"{float(r['AverageNs']) * 1e-3:.2f} | {float(r['Percentage']):.2f} |")
    with open(os.path.join(PROFILE_DIR, "bench_extras_all_kernels_trace.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def reverse_profile_commands(prec: str) -> dict:
    """The rocprofv3 commands behind the reverse-step summaries (bench.py --reverse-only)."""
    d = "gpurun_out" if prec == "f32" else f"gpurun_out/p_{prec}"
    cmd = f"python bench.py --reverse-only --prec {prec}"
    out = {k: f"rocprofv3 --pmc {c} --output-format csv -d {d}/rp_rev_{k} -o rev -- {cmd}"
           for k, c in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE"), ("valu", "VALUBusy"),
                        ("flops", " ".join(flop_counters(prec))))}
    out["trace"] = f"rocprofv3 --kernel-trace --stats --output-format csv -d {d}/rp_rev_trace -o rev -- {cmd}"
    out["copy_fetch"], out["copy_write"] = PROFILE_COMMANDS["copy_fetch"], PROFILE_COMMANDS["copy_write"]
    return out


def reverse_profile_summary(out_root: str, prec: str, n: int = 4096):
    """Kernel trace and counters of the reverse-step kernels (one and two steps per launch) from
    the output of reverse_profile_commands(prec) under out_root (rp_copy_* calibration beside it)."""
    import re

    cmds = reverse_profile_commands(prec)
    d = lambda k: os.path.join(out_root, f"rp_rev_{k}")
    if not os.path.isdir(d("trace")):
        return
    sb, ab = (8, 8) if prec == "f64" else (4, 4)
    cells = n * n
    alg = {"1": cells * (9 * sb + 18 * ab), "2": cells * (18 * sb + 18 * ab)}
    stats = _csv_rows(_find_csv(d("trace"), "kernel_stats.csv"))
    fetch = _csv_rows(_find_csv(d("fetch"), "counter_collection.csv"))
    write = _csv_rows(_find_csv(d("write"), "counter_collection.csv"))
    valu = _csv_rows(_find_csv(d("valu"), "counter_collection.csv"))
    flops = _csv_rows(_find_csv(d("flops"), "counter_collection.csv"))
    cf, _ = _per_dispatch(_csv_rows(_find_csv(os.path.join(out_root, "rp_copy_fetch"), "counter_collection.csv")),
                          "copyBuffer")
    cw, _ = _per_dispatch(_csv_rows(_find_csv(os.path.join(out_root, "rp_copy_write"), "counter_collection.csv")),
                          "copyBuffer")
    gib_kib = (1 << 30) / 1024
    fscale, wscale = gib_kib / cf, gib_kib / cw
    rows = ["| kernel | steps per launch | calls | average us | us per step | HBM bytes (scaled) | / algorithmic "
            "| GB/s at algorithmic bytes | frac of 8 TB/s | VALUBusy % | flops per node and step |",
            "|---|---|---|---|---|---|---|---|---|---|---|"]
    blob = {"prec": prec, "n": n, "algorithmic_bytes": alg, "kernels": {}}
    for r in stats:
        m = re.search(r"k_adjoint_strip([12])<(\d+), (\d+)>", r["Name"])
        if not m:
            continue
        depth, model = m.group(1), int(m.group(2))
        key = f"k_adjoint_strip{depth}<{model}, {m.group(3)}>"
        label = f"k_adjoint_strip{depth}<{MODEL_ORDER[model] if model < 8 else model}, {prec}>"
        avg = float(r["AverageNs"]) * 1e-3
        f_kib, _ = _per_dispatch(fetch, key)
        w_kib, _ = _per_dispatch(write, key)
        hbm = None if f_kib is None or w_kib is None else f_kib * 1024 * fscale + w_kib * 1024 * wscale
        vb, _ = _per_dispatch(valu, key)
        fl = _flops_per_dispatch(flops, key, prec)
        st = int(depth)
        gbs = alg[depth] / (avg * 1e-6) / 1e9
        fpn = None if fl is None else fl / (cells * st)
        rows.append(f"| {label} | {st} | {r['Calls']} | {avg:.1f} | {avg / st:.1f} | "
                    f"{'' if hbm is None else f'{hbm:.4g}'} | {'' if hbm is None else f'{hbm / alg[depth]:.4f}'} | "
                    f"{gbs:.1f} | {gbs / HBM_PEAK_GBS:.4f} | {'' if vb is None else f'{vb:.1f}'} | "
                    f"{'' if fpn is None else f'{fpn:.1f}'} |")
        blob["kernels"][label] = {"avg_us": round(avg, 2), "hbm_bytes": None if hbm is None else int(hbm),
                                  "valu_busy": None if vb is None else round(vb / 100, 4),
                                  "flops_per_node_step": None if fpn is None else round(fpn, 1),
                                  "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
    text = [f"# Adjoint reverse steps ({prec}, {n}x{n} double shear layer states): trace and counters", "",
            "Commands (from the repository root; each counter in a run of its own):", "", "```",
            *(cmds[k] for k in ("trace", "fetch", "write", "valu", "flops", "copy_fetch", "copy_write")), "```", "",
            f"Algorithmic bytes per launch: one reverse step per launch {n}*{n} * (9 s + 18 a) = {alg['1']} B "
            f"(f_n pulled, lambda_n+1 gathered, lambda_n written); two per launch {n}*{n} * (18 s + 18 a) = "
            f"{alg['2']} B (f_n, f_n-1 and lambda_n+1 read, lambda_n-1 written; s = a = {sb} B). HBM bytes: "
            f"FETCH_SIZE x {fscale:.4f} + WRITE_SIZE x {wscale:.4f} (the same 1 GiB copy calibration as the "
            "step-kernel counters). The copy kernel, which reads whole lines, shows half its true bytes in "
            "FETCH_SIZE; requests for parts of lines, which these gathers make at strip edges, need not be "
            "undercounted the same way, so here the scaled figure is an upper bound. Flops: 64 lanes x (ADD + MUL + TRANS + 2 FMA) "
            "VALU instructions per dispatch over the node updates it makes (the two-step kernel's include "
            "its halo).", "", *rows, "",
            "```json", json.dumps(blob, indent=1), "```", ""]
    with open(os.path.join(PROFILE_DIR, f"adjoint_reverse_{prec}_dsl4096.md"), "w") as fh:
        fh.write("\n".join(text))


PROFILE_ARGS = "--steps 40 --warmup 4 --no-cpu --no-extras"
EXTRAS_PROFILE_COMMAND = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/rp_trace_all -o bench -- "
                          "python bench.py --steps 20 --warmup 2 --no-cpu --batch-steps 2000")
PROFILE_COMMANDS = {
    "trace": f"rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/rp_trace -o bench -- "
             f"python bench.py {PROFILE_ARGS}",
    "fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/rp_fetch -o bench -- "
             f"python bench.py {PROFILE_ARGS}",
    "write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/rp_write -o bench -- "
             f"python bench.py {PROFILE_ARGS}",
    "copy_fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/rp_copy_fetch -o copy -- "
                  "python bench.py --copy-probe",
    "copy_write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/rp_copy_write -o copy -- "
                  "python bench.py --copy-probe",
    "valu": f"rocprofv3 --pmc VALUBusy --output-format csv -d gpurun_out/rp_valu -o bench -- "
            f"python bench.py {PROFILE_ARGS}",
    "flops": f"rocprofv3 --pmc {' '.join(flop_counters('f32'))} --output-format csv -d gpurun_out/rp_flops -o bench -- "
             f"python bench.py {PROFILE_ARGS}",
}


def profile_commands(prec: str) -> dict:
    """The rocprofv3 commands whose csv output `--profile-summary` reads, for one precision (FP32:
    PROFILE_COMMANDS; others in a p_<prec> folder beside those outputs, with the FP32 run's copy
    calibration)."""
    if prec == "f32":
        return PROFILE_COMMANDS
    args = f"{PROFILE_ARGS} --prec {prec}"
    d = f"gpurun_out/p_{prec}"
    out = {k: f"rocprofv3 --pmc {c} --output-format csv -d {d}/rp_{k} -o bench -- python bench.py {args}"
           for k, c in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE"), ("valu", "VALUBusy"),
                        ("flops", " ".join(flop_counters(prec))))}
    out["trace"] = (f"rocprofv3 --kernel-trace --stats --output-format csv -d {d}/rp_trace -o bench -- "
                    f"python bench.py {args}")
    out["copy_fetch"], out["copy_write"] = PROFILE_COMMANDS["copy_fetch"], PROFILE_COMMANDS["copy_write"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--prec", default="f32", choices=["f32", "f64", "f16"])
    ap.add_argument("--models", default="BGK,RM,HM,CM,CHM,K,PR,RR")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64/FP16, batched and adjoint measurements")
    ap.add_argument("--batch-steps", type=int, default=20000)
    ap.add_argument("--reverse-only", action="store_true",
                    help="only time the adjoint's reverse steps (one and two per launch) at the bench grid")
    ap.add_argument("--stability-map", type=int, metavar="L",
                    help="only run the stability-domain map on L x L vortices (Section 5b; L = 256 is "
                         "the paper's resolution, minutes of GPU time) and print it as JSON")
    ap.add_argument("--profile-summary", metavar="DIR",
                    help="summarise the rocprofv3 csv output of PROFILE_COMMANDS found under DIR "
                         "into profiles/ (no GPU use)")
    ap.add_argument("--reverse-profile-summary", metavar="DIR",
                    help="summarise the rocprofv3 csv output of reverse_profile_commands(prec) found under "
                         "DIR (with the copy calibration beside it) into profiles/ (no GPU use)")
    args = ap.parse_args()
    if args.reverse_profile_summary:
        reverse_profile_summary(args.reverse_profile_summary, args.prec, args.n)
        return
    if args.profile_summary:
        profile_summary(args.profile_summary, args.prec, args.n, profile_commands(args.prec))
        if args.prec == "f32":
            extras_trace_summary(args.profile_summary, EXTRAS_PROFILE_COMMAND)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the grid would shard as y-slabs with a one-row halo)", file=sys.stderr)
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
    if args.reverse_only:
        nu = inputs.dsl_nu(args.n, 0.1)
        rho, ux, uy = inputs.dsl_fields(args.n, args.n, 0.1)
        out = adjoint_step_rate(args.n, args.models.split(","), rho, ux, uy, inputs.rates(nu, "REG"), args.prec)
        print(json.dumps({"reverse_step": out}), flush=True)
        return
    if args.stability_map:
        L = args.stability_map
        out = stability_map(L=L, check_every=max(64, L), progress_s=30.0)
        print(json.dumps({"stability_map": out}), flush=True)
        return
    models = args.models.split(",")
    n = args.n
    mach = 0.1
    nu = inputs.dsl_nu(n, mach)
    omega = inputs.rates(nu, "REG")
    rho, ux, uy = inputs.dsl_fields(n, n, mach)
    sims = {m: Sim(rho, ux, uy, prec=args.prec, eq_order=4, device="cuda:0") for m in models}
    settle_clocks(0.3, args.prec, n)
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
    # right after the timed region, queued back to back with one synchronisation (an idle gap would
    # let the clocks drop): each model's own launch duration over whole fused launches only (an
    # event between the launches inside the timed region costs ~1.5% of the rate; the leftover
    # launch of a window, two steps of a 20-step window, is not one of these launches), five more
    # windows per model, and the same grid, layout and launches with the collision left out
    lw = fused_launch_windows(sims, models, omega, args.steps)
    rw = repeated_windows(sims, models, omega, args.steps)
    ref_sim = next(iter(sims.values()))
    sspl = launch_steps(ref_sim, "STREAM_ONLY")
    nl = max(4, args.steps // sspl)  # whole fused launches only
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ref_sim.step("STREAM_ONLY", omega, nl * sspl)
    ev1.record()
    torch.cuda.synchronize()
    launch_us = launch_us_from(lw)
    stream_launch_us = ev0.elapsed_time(ev1) * 1e3 / nl

    cells = n * n
    bpc = bytes_per_cell(args.prec)
    per_model = {}
    for m in models:
        ms = ev[m][0].elapsed_time(ev[m][1])
        ring, strip = sims[m].fusion(m)
        spl = launch_steps(sims[m], m)
        mlups = cells * args.steps / (ms * 1e-3) / 1e6
        gbs = mlups * 1e6 * bpc / spl / 1e9
        per_model[m] = {"mlups": round(mlups, 1), "us_per_step": round(ms * 1e3 / args.steps, 2),
                        "steps_per_launch": spl, "ring_rows": ring, "strip_rows": strip,
                        "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                        "launch_us": round(launch_us[m], 2)}
    status = {m: s.status() for m, s in sims.items()}
    repeats = repeats_from(rw, cells, args.steps)
    # last: its restoring lbm_set_fusion drops the contexts' two-step tail shape
    single = single_step_rates(sims, models, omega, cells, bpc, max(10, args.steps // 10))
    value = cells * args.steps * len(models) / wall / 1e6
    dominant = max(models, key=lambda m: per_model[m]["launch_us"])  # the slowest kernel
    spl = per_model[dominant]["steps_per_launch"]
    dom_launch_us = per_model[dominant]["launch_us"]
    kname = {3: "k_step3n" if args.prec == "f64" else "k_step3", 2: "k_step2", 1: "k_step"}[spl]
    for m in models:
        rec = counter_record(m, args.prec) if n == 4096 else None
        lu = per_model[m]["launch_us"]
        mf = None if rec is None else rec["hbm_bytes"] / (lu * 1e-6) / 1e9 / HBM_PEAK_GBS
        per_model[m]["valu_busy"] = None if rec is None else rec.get("valu_busy")
        per_model[m]["limiter"] = limiter(rec, mf)
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
        "roofline": roofline_block(dominant, args.prec, kname, cells, bpc, spl, dom_launch_us, stream_launch_us, n),
        "single_step": single,
        "per_model": per_model,
        "repeats": repeats,
        "blowup": {m: st[1] for m, st in status.items()},
    }
    for s in sims.values():
        s.close()
    del sims
    torch.cuda.empty_cache()
    if not args.no_extras:
        fields = (rho, ux, uy)
        extra_steps = max(20, args.steps // 2)
        note("other precisions")
        line["precisions"] = {p: time_models(p, n, models, extra_steps, 5, omega, fields) for p in ("f64", "f16")}
        note("cache-resident grids")
        line["small_grids"] = cache_resident_rates(models)
        # the same grids under the SRT preset (one rate for every non-conserved moment)
        note("SRT preset")
        srt = inputs.rates(nu, "SRT")
        line["srt_preset"] = {"omega": [round(w, 6) for w in srt],
                              "mlups": {m: v["mlups"] for m, v in
                                        time_models(args.prec, n, models, extra_steps, 5, srt, fields).items()}}
        release_settle()
        f64_mlups = min(v["mlups"] for v in line["precisions"]["f64"].values())
        note("batched sweep")
        line["batched"] = batched_sweep(args.batch_steps, f64_mlups)
        note("adjoint")
        line["adjoint"] = adjoint_run()
        line["adjoint"]["reverse_step"] = adjoint_step_rate(n, models, rho, ux, uy, omega)
        note("precision errors")
        line["precision_error"] = precision_errors(n)
        note("stability map")
        line["stability_map"] = stability_map()
        note("double shear layer study")
        line["dsl_study"] = dsl_study()
        note("transport study")
        line["transport_study"] = transport_study()
        note("linear stability domain")
        line["lsa_domain"] = lsa_domain()
    if not args.no_cpu:
        note("oracle on the host cores")
        line["cpu_baseline"] = cpu_baseline(models)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
