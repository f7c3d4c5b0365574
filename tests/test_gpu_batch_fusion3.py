"""Three steps per pass of the batched persistent kernel (lbm_batch_set_fusion_depth 3) against the
plain kernel: live instances stay bit-identical, blow-up steps are the same, retired instances
keep the state of their retirement step, for run lengths that are and are not multiples of three
(the remainder takes single steps), strips wider than the grid, FP64 and FP32; autotuning may pick
it and leaves states, counters and blow-up records unchanged.
"""
import numpy as np
import pytest
import torch

from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.batch import Batch
from paper_2002_05265_amd.binding import LbmError

from test_gpu_batch_fusion import fields_of, make_instances, plain

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,strip", [("f64", 16), ("f32", 8)])
def test_three_steps_bit_identical_to_plain(gpu, prec, strip):
    rng = np.random.default_rng(27)
    insts = make_instances(rng)
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    b = Batch(insts, fields, prec=prec, device=gpu)
    b.set_fusion(strip)
    b.set_fusion_depth(3)
    assert (b.fusion(), b.fusion_depth()) == (strip, 3)
    for k in (13, 4, 2, 18):  # 37 steps: triples and single remainders
        b.run(k)
    step, blow = b.status()
    assert step == 37
    for k, d in enumerate(insts):
        print(f"three-step batch {prec} strip {strip} instance {k} {d['model']} {d['nx']}x{d['ny']}", flush=True)
        ref, st = plain(d, fields[k], prec, 37, gpu)
        np.testing.assert_array_equal(b.state(k).cpu().numpy(), ref)
        assert blow[k] == st[1]
    b.close()


def test_three_steps_blowup_and_retire(gpu):
    rng = np.random.default_rng(28)
    insts = make_instances(rng, n=8, sizes=[(64, 64), (130, 70)])
    # an unstable instance (BGK, second-order equilibrium, Ma 0.5, nu 1e-7, velocity noise)
    insts[3] = {"nx": 64, "ny": 64, "model": "BGK", "eq_order": 2, "omega": list(inputs.rates(1e-7, "SRT")),
                "rho0": 1.0, "mach": 0.5}
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    noise = np.random.default_rng(5)
    r3, u3, v3 = fields[3]
    fields[3] = (r3, u3 + 0.05 * noise.standard_normal(u3.shape), v3 + 0.05 * noise.standard_normal(v3.shape))
    b = Batch(insts, fields, device=gpu)
    b.set_fusion(16)
    b.set_fusion_depth(3)
    b.run(41)
    act = torch.ones(len(insts), dtype=torch.int32, device=gpu)
    act[1] = 0
    act[6] = 0
    b.set_active(act)
    b.run(173)
    b.run(187)
    step, blow = b.status()
    assert step == 401
    _, st = plain(insts[3], fields[3], "f64", 401, gpu)
    assert st[1] >= 0 and blow[3] == st[1], (blow[3], st)
    for k, d in enumerate(insts):
        if k == 3:
            continue
        steps = 41 if k in (1, 6) else 401
        print(f"three-step batch instance {k} after {steps} steps", flush=True)
        ref, stk = plain(d, fields[k], "f64", steps, gpu)
        np.testing.assert_array_equal(b.state(k).cpu().numpy(), ref)
        assert blow[k] == stk[1]
    b.close()


def test_three_steps_autotune_and_validation(gpu):
    rng = np.random.default_rng(29)
    insts = make_instances(rng, n=10, sizes=[(128, 128), (200, 96)])
    fields = [fields_of(d, k) for k, d in enumerate(insts)]
    want = Batch(insts, fields, device=gpu)
    want.set_fusion(0)
    want.run(29)
    ref = [want.state(k).cpu().numpy() for k in range(len(insts))]
    ref_blow = want.status()[1]
    want.close()
    b = Batch(insts, fields, device=gpu)
    b.run(5)
    blow0 = b.status()[1]
    npt, gpc, us = b.autotune(2)
    print(f"autotune: npt {npt} gpc {gpc} fusion {b.fusion()} depth {b.fusion_depth()} {us:.1f} us/step", flush=True)
    assert npt in (1, 2, 4) and gpc >= 1 and us > 0 and b.fusion() in (0, 64) and b.fusion_depth() in (2, 3)
    step, blow = b.status()  # the timed passes ran ahead of the counter: records as they were
    assert step == 5 and list(blow) == list(blow0)
    b.set_fusion(16)  # a strip height other than the autotuned one: the tables are re-dealt
    b.set_fusion_depth(3)
    b.run(24)
    step, blow = b.status()
    assert step == 29 and list(blow) == list(ref_blow)
    for k in range(len(insts)):
        np.testing.assert_array_equal(b.state(k).cpu().numpy(), ref[k])
    for bad in (0, 1, 4):
        with pytest.raises(LbmError):
            b.set_fusion_depth(bad)
    b.close()
    h = Batch(insts[:2], fields[:2], prec="f16", device=gpu)
    with pytest.raises(LbmError):
        h.set_fusion_depth(3)
    assert h.fusion_depth() == 2
    h.close()
