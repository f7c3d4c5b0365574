"""Two steps per pass of the batched persistent kernel (lbm_batch_set_fusion) against the plain
kernel: live instances stay bit-identical, blow-up steps are the same, retired instances keep
the state of their retirement step, and |u|^2 means agree, for runs whose lengths are and are not
multiples of four (the remainder takes single steps), strips wider than the grid, all three
precisions, and autotuning that may switch two steps per pass on or off.
"""
import numpy as np
import pytest
import torch

from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.batch import Batch
from paper_2002_05265_amd.sim import Sim

pytestmark = pytest.mark.gpu

SIZES = [(64, 64), (96, 40), (37, 23), (128, 130), (70, 45), (256, 64), (2, 9)]


def make_instances(rng, n=14, sizes=SIZES):
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
    return inputs.fourier_mode_fields(inst["nx"], inst["ny"], inst["mach"], np.random.default_rng(200 + k),
                                      amplitude=2e-2)


def plain(inst, fields, prec, steps, gpu):
    s = Sim(*fields, prec=prec, eq_order=inst["eq_order"], device=gpu,
            ref_velocity=(inst.get("ux0", 0.0), inst.get("uy0", 0.0)))
    s.step(inst["model"], inst["omega"], steps)
    out, st = s.state().cpu().numpy(), s.status()
    s.close()
    return out, st


@pytest.mark.parametrize("prec,strip", [("f64", 16), ("f32", 8), ("f16", 24)])
def test_bit_identical_to_plain(gpu, prec, strip):
    rng = np.random.default_rng(17)
    insts = make_instances(rng)
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    b = Batch(insts, fields, prec=prec, device=gpu)
    b.set_fusion(strip)
    assert b.fusion() == strip
    for k in (13, 4, 2, 18):  # 37 steps: pairs and single remainders
        b.run(k)
    step, blow = b.status()
    assert step == 37
    for k, d in enumerate(insts):
        print(f"fused batch {prec} strip {strip} instance {k} {d['model']} {d['nx']}x{d['ny']}", flush=True)
        ref, st = plain(d, fields[k], prec, 37, gpu)
        np.testing.assert_array_equal(b.state(k).cpu().numpy(), ref)
        assert blow[k] == st[1]
    b.close()


def test_blowup_retire_and_mean_u2(gpu):
    rng = np.random.default_rng(18)
    insts = make_instances(rng, n=8, sizes=[(64, 64), (130, 70)])
    # an unstable instance (BGK, second-order equilibrium, Ma 0.5, nu 1e-7, velocity noise)
    insts[3] = {"nx": 64, "ny": 64, "model": "BGK", "eq_order": 2, "omega": list(inputs.rates(1e-7, "SRT")),
                "rho0": 1.0, "mach": 0.5}
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    noise = np.random.default_rng(5)
    r3, u3, v3 = fields[3]
    fields[3] = (r3, u3 + 0.05 * noise.standard_normal(u3.shape), v3 + 0.05 * noise.standard_normal(v3.shape))
    a = Batch(insts, fields, device=gpu)
    b = Batch(insts, fields, device=gpu)
    b.set_fusion(16)
    for x in (a, b):
        x.run(40)
    ua, ub = a.mean_u2().clone(), b.mean_u2().clone()
    live = torch.tensor([k != 3 for k in range(len(insts))], device=gpu)
    assert torch.equal(ua[live], ub[live])
    # retire instances 1 and 6 at step 40, then run on to 400 (past the blow-up of instance 3)
    act = torch.ones(len(insts), dtype=torch.int32, device=gpu)
    act[1] = 0
    act[6] = 0
    for x in (a, b):
        x.set_active(act)
        x.run(173)
        x.run(187)
    (sa, ba), (sb, bb) = a.status(), b.status()
    assert sa == sb == 400
    _, st = plain(insts[3], fields[3], "f64", 400, gpu)
    assert st[1] >= 0 and ba[3] == bb[3] == st[1], (ba[3], bb[3], st)
    for k, d in enumerate(insts):
        if k == 3:
            continue
        steps = 40 if k in (1, 6) else 400
        ref, stk = plain(d, fields[k], "f64", steps, gpu)
        np.testing.assert_array_equal(b.state(k).cpu().numpy(), ref)
        np.testing.assert_array_equal(a.state(k).cpu().numpy(), ref)
        assert bb[k] == ba[k] == stk[1]
    a.close()
    b.close()


def test_autotune_and_validation(gpu):
    rng = np.random.default_rng(19)
    insts = make_instances(rng, n=10, sizes=[(128, 128), (200, 96)])
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    want = Batch(insts, fields, device=gpu)
    want.run(29)
    ref = [want.state(k).cpu().numpy() for k in range(len(insts))]
    want.close()
    b = Batch(insts, fields, device=gpu)
    b.run(5)
    npt, gpc, us = b.autotune(2)
    print(f"autotune: npt {npt} gpc {gpc} fusion {b.fusion()} {us:.1f} us/step", flush=True)
    assert npt in (1, 2, 4) and gpc >= 1 and us > 0 and b.fusion() in (0, 64)
    assert b.status()[0] == 5
    b.run(24)
    for k in range(len(insts)):
        np.testing.assert_array_equal(b.state(k).cpu().numpy(), ref[k])
    for bad in (-8, 4, 12):
        with pytest.raises(RuntimeError):
            b.set_fusion(bad)
    b.set_fusion(0)
    assert b.fusion() == 0
    b.close()
