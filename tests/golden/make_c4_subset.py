"""Write tests/golden/c4_subset.npz: the oracle's runs of a stratified subset of the batched
stability sweep (two instances per collision model on 64 x 64 grids, Ma ~ U[0, 0.6],
log10 nu ~ U[-7, -2], SRT and REG in turn, one random Fourier-mode perturbation of amplitude
1e-3 each, extended equilibrium), over the sweep's full 20000 steps.

Stored per instance: its parameters; the first step whose state has a node with !(rho > 0)
(-1 if none up to step 20000); for runs that stay positive, the FP64 totals of the final state
and the final populations at 256 seeded nodes.  Also NPERT runs in which every population is
perturbed by ULPS ulps (relative 64 x 2^-52) after every step, random signs drawn anew per step
and run: a model of the rounding differences between two FP64 implementations of the same
collision, whose ~200 roundings per node in a different order and with or without fused
multiply-adds differ by up to tens of ulps per population and step.  Stored: their blow-up steps
(how far rounding alone moves the blow-up of this run) and, where all stay positive, the largest
relative change of the final state and the largest change of each total (the trajectory's
sensitivity to rounding).

For a run that blows up in any of these, also its state half-way to the earliest blow-up, where
the trajectories still agree, and the perturbed runs' largest relative change there.

Each initial field is one Fourier mode (kx, ky), so it is constant along the lines of constant
phase kx i / nx + ky j / ny, and any arithmetic that treats every node alike keeps it so (the
oracle's and the GPU's included).  The perturbations therefore draw their signs per population
and phase line: they do not seed the transverse modes that no rounding difference can seed (a
per-node random perturbation does, and blows some stable runs up).

Calls only the oracle and the input generators.  Runs the instances in parallel processes (a few
minutes on 8 cores).

    python tests/golden/make_c4_subset.py
"""
import multiprocessing as mp
import pathlib
import sys
import time

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from paper_2002_05265_amd import inputs  # noqa: E402

STEPS, CHUNK, NSAMPLE, NPERT = 20000, 100, 256, 3
ULPS = 64  # perturbation per population and step, in units of 2^-52 (relative)
OUT = pathlib.Path(__file__).with_name("c4_subset.npz")


def bad(f):
    return not bool(np.all(f.sum(axis=0) > 0.0))


def run_to_blowup(f, code, omega, steps):
    """(final state, first step n in [0, steps] whose state is bad, -1 if none)."""
    n = 0
    while n < steps:
        k = min(CHUNK, steps - n)
        g = oracle.step(f, code, 4, omega, k)
        if bad(f) or bad(g):  # find the first bad state of this chunk step by step
            h = f
            for j in range(k + 1):
                if bad(h):
                    return h, n + j
                h = oracle.step(h, code, 4, omega, 1)
        f, n = g, n + k
    return f, (steps if bad(f) else -1)


def run_perturbed(f0, code, omega, line, seed, steps):
    """(final state, blow-up step) with a perturbation of ULPS ulps of every population after every
    step, signs per population and phase line."""
    rng = np.random.default_rng(seed)
    f = f0
    for n in range(steps):
        if bad(f):
            return f, n
        signs = rng.choice([-1.0, 1.0], size=(9, line.max() + 1))
        f = oracle.step(f, code, 4, omega, 1) * (1.0 + signs[:, line] * (ULPS * 2.0 ** -52))
    return f, (steps if bad(f) else -1)


def run(d):
    t = time.time()
    code = inputs.MODEL_CODES[d["model"]]
    fields = inputs.sweep_fields(d)
    f0 = oracle.init_eq(4, *fields)
    f, blow = run_to_blowup(f0, code, d["omega"], STEPS)
    kx, ky = inputs.sweep_mode(d)
    i = np.arange(d["nx"])[None, :]
    j = np.arange(d["ny"])[:, None]
    # phase line of each node (the fields depend on (i, j) only through it), numbered densely
    _, line = np.unique(np.mod(kx * i * d["ny"] + ky * j * d["nx"], d["nx"] * d["ny"]), return_inverse=True)
    line = line.reshape(-1)
    pert = [run_perturbed(f0, code, d["omega"], line.reshape(d["ny"], d["nx"]),
                          s, STEPS) for s in range(NPERT)]
    out = {"blowup": blow, "perturbed_blowup": [b for _, b in pert]}
    finite = [b for b in (blow, *out["perturbed_blowup"]) if b >= 0]
    idx = np.random.default_rng(100 + d["index"]).choice(d["nx"] * d["ny"], NSAMPLE, replace=False)
    out["nodes"] = idx
    if finite:
        # an unstable run: its state half-way to the earliest blow-up of any run, where the
        # trajectories still agree, and their spread there
        mid = min(finite) // 2
        fm = oracle.step(f0, code, 4, d["omega"], mid)
        gm = [run_perturbed(f0, code, d["omega"], line.reshape(d["ny"], d["nx"]), s, mid)[0] for s in range(NPERT)]
        out["mid_step"] = mid
        out["mid_f"] = fm.reshape(9, -1)[:, idx]
        out["mid_sensitivity"] = max(float(np.max(np.abs(g - fm)) / np.max(np.abs(fm))) for g in gm)
    if blow < 0:
        stable = all(b < 0 for _, b in pert)
        out["sensitivity"] = (max(float(np.max(np.abs(g - f)) / np.max(np.abs(f))) for g, _ in pert)
                              if stable else np.inf)
        out["totals"] = oracle.moments(f)[3]
        tp = [oracle.moments(g)[3] for g, _ in pert]
        out["totals_spread"] = (np.max([np.abs(t - out["totals"]) for t in tp], axis=0)
                                if stable else np.full(5, np.inf))
        out["f"] = f.reshape(9, -1)[:, idx]
    print(f"{d['index']:2d} {d['model']:3s} {d['preset']} Ma {d['mach']:.3f} nu {d['nu']:.2e}: "
          f"blow-up {blow}, perturbed {out['perturbed_blowup']}, "
          f"sensitivity {out.get('sensitivity', 0):.1e}, {time.time() - t:.0f} s", flush=True)
    return out


if __name__ == "__main__":
    oracle.build()
    insts = inputs.stratified_sweep_instances()
    with mp.Pool(8) as pool:
        res = pool.map(run, insts)
    data = {"steps": np.array(STEPS), "ulps": np.array(ULPS),
            "mach": np.array([d["mach"] for d in insts]), "nu": np.array([d["nu"] for d in insts]),
            "blowup": np.array([r["blowup"] for r in res]),
            "perturbed_blowup": np.array([r["perturbed_blowup"] for r in res])}
    for k, r in enumerate(res):
        data[f"{k}_nodes"] = np.asarray(r["nodes"])
        for key in ("sensitivity", "totals", "totals_spread", "f", "mid_step", "mid_f", "mid_sensitivity"):
            if key in r:
                data[f"{k}_{key}"] = np.asarray(r[key])
    np.savez_compressed(OUT, **data)
    print("wrote", OUT)
