"""Write tests/golden/c2_profiles.npz: oracle vortex-core profiles of the 1024 x 1024 convected
vortex (Ma = 0.2, beta = 0.15, R = 0.1 L, nu = 1e-6, REG rates, extended equilibrium) at step
1000, and at step 200 (before any model has lost positivity), for the eight collision models.

Profiles: rho - 1 and uy along the row j = L/2, and ux along the column through the
analytically advected centre x = round(L/2 + u0 n) mod L.  Also stored per model: the first
step whose state has a node with !(rho > 0) (-1 if none up to step 1000).  Calls only the oracle and the input
generators.  Runs the eight models in parallel processes (about 10 minutes on 8 cores).

    python tests/golden/make_c2_profiles.py
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

L, MACH, NU, STEPS, EARLY = 1024, 0.2, 1e-6, 1000, 200
OUT = pathlib.Path(__file__).with_name("c2_profiles.npz")


def column(nsteps=STEPS):
    return int(round(L / 2 + MACH * inputs.CS * nsteps)) % L


def bad(f):
    rho = f.sum(axis=0)
    return not bool(np.all(rho > 0.0))


def run(name):
    t = time.time()
    rho, ux, uy = inputs.vortex_fields(L, L, MACH, beta=0.15, radius_frac=0.1)
    f = oracle.init_eq(4, rho, ux, uy)
    blowup = -1  # first step n in [0, STEPS] whose state has a node with !(rho > 0)
    early = None
    for n in range(STEPS):
        if blowup < 0 and bad(f):
            blowup = n
        if n == EARLY:
            r, u, v, _ = oracle.moments(f)
            early = np.stack([r[L // 2, :] - 1.0, v[L // 2, :], u[:, column(EARLY)]])
        f = oracle.step(f, oracle.MODELS[name], 4, inputs.rates(NU, "REG"), 1)
    if blowup < 0 and bad(f):
        blowup = STEPS
    r, u, v, tot = oracle.moments(f)
    c = column()
    print(f"{name}: {time.time() - t:.0f} s, blow-up step {blowup}", flush=True)
    return name, np.stack([r[L // 2, :] - 1.0, v[L // 2, :], u[:, c]]), tot, blowup, early


if __name__ == "__main__":
    oracle.build()
    with mp.Pool(8) as pool:
        res = pool.map(run, list(oracle.MODELS))
    data = {f"{n}_profiles": p for n, p, _, _, _ in res}
    data.update({f"{n}_totals": t for n, _, t, _, _ in res})
    data.update({f"{n}_blowup": np.array(b) for n, _, _, b, _ in res})
    data.update({f"{n}_profiles_{EARLY}": e for n, _, _, _, e in res})
    data["column"] = np.array(column())
    data[f"column_{EARLY}"] = np.array(column(EARLY))
    data["early_step"] = np.array(EARLY)
    np.savez_compressed(OUT, **data)
    print("wrote", OUT)
