"""The batched sweep captured in a HIP graph: lbm_batch_run on the batch's stream inside a stream
capture (torch.cuda.CUDAGraph), then replayed.  The persistent kernels take the step from the
device counter, so every replay advances every instance as a direct run does: blow-up steps,
states and the domain means of |u|^2 after each replay equal those of a batch advanced by direct
calls, bit for bit.  Replays are separated by eager work and synchronisations of the program."""
import numpy as np
import pytest
import torch

from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.batch import Batch

pytestmark = pytest.mark.gpu


def instances():
    rng = np.random.default_rng(31)
    insts = []
    for k, model in enumerate(list(inputs.MODEL_NAMES) * 2):
        n = [48, 64, 100][k % 3]
        insts.append({"nx": n, "ny": n + 8 * (k % 2), "model": model, "eq_order": 4,
                      "omega": list(inputs.rates(10 ** rng.uniform(-6, -3), "REG" if k % 2 else "SRT")),
                      "rho0": 1.0, "mach": float(rng.uniform(0.1, 0.6)), "field_seed": 500 + k})
    return insts


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_graph_replay_matches_direct_runs(gpu, prec):
    insts = instances()
    fields = [inputs.fourier_mode_fields(d["nx"], d["ny"], d["mach"], np.random.default_rng(d["field_seed"]))
              for d in insts]
    s = torch.cuda.Stream()
    direct = Batch(insts, fields, prec=prec, device=gpu)
    b = Batch(insts, fields, prec=prec, device=gpu, stream=s)
    steps = 10  # three steps per pass and a single step: both launch shapes
    direct.run(steps)
    b.run(steps)  # probes the residency of both shapes before the capture
    s.synchronize()
    torch.cuda.synchronize()
    print(f"graph {prec}: capturing lbm_batch_run({steps})", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.run(steps)
    assert b.status()[0] == steps  # capturing ran nothing
    for r in range(4):
        g.replay()
        # eager work of the program between replays
        x = torch.randn(4096, device=gpu)
        assert torch.isfinite(x.sum()).item()
        s.synchronize()
        direct.run(steps)
        sb, bb = b.status()
        sd, bd = direct.status()
        print(f"  replay {r}: step {sb} / {sd}, blow-ups {sum(v >= 0 for v in bb)}", flush=True)
        assert sb == sd == steps * (r + 2)
        assert bb == bd
        ub, ud = b.mean_u2(), direct.mean_u2()
        torch.cuda.synchronize()
        assert torch.equal(ub, ud)
        for k in range(len(insts)):
            assert torch.equal(b.state(k), direct.state(k)), (r, k)
    b.close()
    direct.close()
