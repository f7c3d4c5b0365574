"""Batched persistent sweep (include/lbm_batch.h) against the plain kernel and the oracle.

- Bit-identity: every instance of a batch equals the same run through lbm_init / lbm_step,
  for every model, equilibrium order, uneven grid sizes and all three precisions.
- Blow-up steps equal those of the plain kernel; a NaN injected into one instance's initial
  fields flags that instance at step 0 and leaves every other instance bit-identical.
- Autotuning, chunked runs and re-dealing the live instances over the XCDs leave the results
  unchanged.
- A stratified subset (every model, small grids) matches the oracle (FP64 within 1e-12, or
  the same blow-up step within one step).  Random sweep parameters include linearly unstable
  runs that have not yet lost positivity; there rounding-level differences grow step by step,
  so the bar is max(1e-12, 64 x the trajectory's own sensitivity), the sensitivity being the
  oracle's response to a one-ulp relative perturbation of the initial populations.
"""
import numpy as np
import pytest

import oracle
from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.batch import Batch
from paper_2002_05265_amd.sim import Sim

pytestmark = pytest.mark.gpu

SIZES = [(64, 64), (96, 40), (37, 23), (128, 130), (70, 45), (256, 64)]


def make_instances(rng, n=16, sizes=SIZES):
    out = []
    for k in range(n):
        nx, ny = sizes[k % len(sizes)]
        model = inputs.MODEL_NAMES[k % 8]
        N = 4 if model in ("CM", "CHM", "K") else int(rng.choice([2, 3, 4]))
        omega = [1.96, *rng.uniform(0.5, 1.9, 4)] if k % 3 else list(inputs.rates(1e-4, "REG"))
        mach = float(rng.uniform(0.05, 0.4))
        out.append({"nx": nx, "ny": ny, "model": model, "eq_order": N, "omega": omega, "rho0": 1.0,
                    "ux0": mach * inputs.CS if k % 2 else 0.0, "uy0": 0.01 * (k % 3), "mach": mach})
    return out


def fields_of(inst, k):
    return inputs.fourier_mode_fields(inst["nx"], inst["ny"], inst["mach"], np.random.default_rng(100 + k),
                                      amplitude=2e-2)


def plain_state(inst, fields, prec, steps, gpu):
    s = Sim(*fields, prec=prec, eq_order=inst["eq_order"], device=gpu,
            ref_velocity=(inst.get("ux0", 0.0), inst.get("uy0", 0.0)))
    s.step(inst["model"], inst["omega"], steps)
    out, st = s.state().cpu().numpy(), s.status()
    s.close()
    return out, st


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_batch_bit_identical_to_plain(gpu, prec):
    rng = np.random.default_rng(7)
    insts = make_instances(rng)
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    b = Batch(insts, fields, prec=prec, device=gpu)
    steps = 37
    b.run(steps)
    step, blow = b.status()
    assert step == steps
    for k, d in enumerate(insts):
        print(f"batch {prec} instance {k} {d['model']} {d['nx']}x{d['ny']}", flush=True)
        ref, st = plain_state(d, fields[k], prec, steps, gpu)
        np.testing.assert_array_equal(b.state(k).cpu().numpy(), ref)
        assert blow[k] == st[1]
    b.close()


def test_batch_shapes_and_chunks_agree(gpu):
    rng = np.random.default_rng(8)
    insts = make_instances(rng, n=10)
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    ref = Batch(insts, fields, device=gpu)
    ref.run(24)
    want = [ref.state(k).cpu().numpy() for k in range(len(insts))]
    ref.close()
    for npt, gpc in [(1, 0), (2, 0), (4, 1), (2, 3)]:
        b = Batch(insts, fields, device=gpu)
        b.set_launch(npt, gpc)
        b.run(10)
        b.run(14)
        assert b.status()[0] == 24
        for k in range(len(insts)):
            np.testing.assert_array_equal(b.state(k).cpu().numpy(), want[k])
        b.close()
    # re-dealing the instances over the XCDs between pieces of a run changes nothing
    b = Batch(insts, fields, device=gpu)
    b.run(24, rebalance_every=5)
    assert b.status()[0] == 24
    for k in range(len(insts)):
        np.testing.assert_array_equal(b.state(k).cpu().numpy(), want[k])
    b.close()
    b = Batch(insts, fields, device=gpu)
    b.run(5)
    npt, gpc, us = b.autotune(3)
    assert npt in (1, 2, 4) and gpc >= 1 and us > 0
    assert b.status()[0] == 5
    b.run(19)
    for k in range(len(insts)):
        np.testing.assert_array_equal(b.state(k).cpu().numpy(), want[k])
    b.close()


def test_batch_blowup_and_nan_isolation(gpu):
    rng = np.random.default_rng(9)
    insts = make_instances(rng, n=8, sizes=[(64, 64)])
    # an unstable instance: BGK with the second-order equilibrium, Ma 0.5, nu 1e-7, white
    # velocity noise of amplitude 0.05 (the oracle loses positivity at step 72)
    insts[3] = {"nx": 64, "ny": 64, "model": "BGK", "eq_order": 2, "omega": list(inputs.rates(1e-7, "SRT")),
                "rho0": 1.0, "mach": 0.5}
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    noise = np.random.default_rng(5)
    r3, u3, v3 = fields[3]
    fields[3] = (r3, u3 + 0.05 * noise.standard_normal(u3.shape), v3 + 0.05 * noise.standard_normal(v3.shape))
    steps = 400
    b = Batch(insts, fields, device=gpu)
    b.run(steps)
    _, blow = b.status()
    _, st = plain_state(insts[3], fields[3], "f64", steps, gpu)
    assert st[1] >= 0 and blow[3] == st[1], (blow[3], st)
    f, ob = oracle.init_eq(2, *fields[3]), -1
    for n in range(steps):
        if not np.all(f.sum(axis=0) > 0):
            ob = n
            break
        f = oracle.step(f, oracle.BGK, 2, insts[3]["omega"], 1)
    assert abs(blow[3] - ob) <= 1, (blow[3], ob)
    clean = [b.state(k).cpu().numpy() for k in range(len(insts))]
    b.close()
    bad = [tuple(np.array(a) for a in f) for f in fields]
    bad[5][1][10, 20] = np.nan
    b2 = Batch(insts, bad, device=gpu)
    b2.run(steps, rebalance_every=50)  # the blown-up instances leave the work lists
    _, blow2 = b2.status()
    assert blow2[5] == 0
    for k in range(len(insts)):
        if k not in (3, 5):
            np.testing.assert_array_equal(b2.state(k).cpu().numpy(), clean[k])
            assert blow2[k] == blow[k]
    assert blow2[3] == blow[3]
    b2.close()


def test_batch_oracle_subset(gpu):
    rng = np.random.default_rng(10)
    insts = []
    for k, model in enumerate(list(inputs.MODEL_NAMES) * 2):
        n = [32, 48][k // 8]
        insts.append({"nx": n, "ny": n + 3 * (k % 3), "model": model, "eq_order": 4,
                      "omega": list(inputs.rates(10 ** rng.uniform(-6, -3), "REG" if k % 2 else "SRT")),
                      "rho0": 1.0, "mach": float(rng.uniform(0.1, 0.5))})
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    steps = 300
    b = Batch(insts, fields, device=gpu)
    b.run(steps)
    _, blow = b.status()
    for k, d in enumerate(insts):
        f = oracle.init_eq(4, *fields[k])
        ob = -1
        for n in range(steps):
            if ob < 0 and not np.all(f.sum(axis=0) > 0):
                ob = n
            f = oracle.step(f, inputs.MODEL_CODES[d["model"]], 4, d["omega"], 1)
        if ob < 0 and not np.all(f.sum(axis=0) > 0):
            ob = steps
        print(f"oracle subset {k} {d['model']} blow-up gpu {blow[k]} oracle {ob}", flush=True)
        if ob >= 0 or blow[k] >= 0:
            assert abs(blow[k] - ob) <= 1
        else:
            g = b.state(k).cpu().numpy()
            err = np.max(np.abs(g - f)) / np.max(np.abs(f))
            sens = trajectory_sensitivity(fields[k], d, steps, f)
            print(f"    error {err:.3e}, sensitivity {sens:.3e}", flush=True)
            assert err < max(1e-12, 64 * sens), (k, err, sens)
    b.close()


def trajectory_sensitivity(fields, d, steps, f_ref):
    """Relative change of the oracle's state after `steps` when every initial population is
    perturbed by one ulp (relative 2^-52, random sign)."""
    f0 = oracle.init_eq(4, *fields)
    sign = np.random.default_rng(0).choice([-1.0, 1.0], size=f0.shape)
    g = oracle.step(f0 * (1.0 + sign * 2.0 ** -52), inputs.MODEL_CODES[d["model"]], 4, d["omega"], steps)
    return float(np.max(np.abs(g - f_ref)) / np.max(np.abs(f_ref)))


def test_full_sweep_bit_identical_to_plain(gpu):
    """The bench's 512-instance random sweep (sides 64..512, every model, SRT and REG alternating),
    autotuned and re-dealt over the XCDs, against each instance's plain run, after 120 steps."""
    import torch

    insts = inputs.sweep_instances(512)
    for k, d in enumerate(insts):
        d["omega"] = inputs.rates(d["nu"], "SRT" if k % 2 == 0 else "REG")
        d["eq_order"] = 4
    fields = [inputs.sweep_fields(d) for d in insts]
    b = Batch(insts, fields, prec="f64", device=gpu)
    b.autotune(2)
    steps = 120
    b.run(steps, rebalance_every=40)
    _, blow = b.status()
    for k, d in enumerate(insts):
        s = Sim(*fields[k], prec="f64", eq_order=4, device=gpu)
        s.step(d["model"], d["omega"], steps)
        st = s.status()[1]
        same = torch.equal(b.state(k), s.state()) if blow[k] < 0 else True
        s.close()
        assert blow[k] == st and same, (k, d["model"], d["nx"], blow[k], st)
    b.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_residency_from_resources(gpu, prec):
    """Every persistent launch shape is sized from its kernel's own resources (VGPRs, SGPR bound,
    LDS, threads) and the runtime's occupancy figure, and the bounded residency probe of its first
    run confirms that size (no step down)."""
    rng = np.random.default_rng(5)
    insts = [{"nx": 64 + 16 * (k % 3), "ny": 64, "model": m, "eq_order": 4,
              "omega": list(inputs.rates(1e-4, "REG")), "rho0": 1.0, "mach": float(rng.uniform(0.1, 0.4))}
             for k, m in enumerate(list(inputs.MODEL_NAMES) * 2)]
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    b = Batch(insts, fields, prec=prec, device=gpu)
    b.autotune(1)  # times every launch shape, probing each one's residency first
    shapes = range(5) if prec != "f16" else range(4)
    for shape in shapes:
        fit, occ, res, down = b.residency(shape)
        print(f"residency {prec} shape {shape}: resources {fit}, runtime {occ}, confirmed {res}", flush=True)
        assert fit >= 1 and res == min(fit, occ), (shape, fit, occ, res)
    assert b.residency(0)[3] == 0  # no probe had to lower a figure
    b.close()
