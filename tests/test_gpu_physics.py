"""The HIP path on random cells and on the physics the oracle is pinned to.

- Collision on 10^6 random cells (positive populations near moving equilibria, density and
  velocity spread, 5% noise): one step (the single-step kernel) against the oracle within 1e-13,
  and one three-step launch (the default on this grid) within 1e-12, in FP64, for every model and
  equilibrium order.
- Shear-wave decay (Section 2's viscosity nu = cs^2 (1/omega - 1/2), no Mach error with the
  fourth-order equilibrium) and the acoustic speed cs = 1/sqrt(3), measured on the GPU in FP64 and
  shifted FP32 (mean-flow reference for the shear wave), within the 0.5% the oracle's own pins
  reach on the same runs.
"""
import numpy as np
import pytest

import oracle
from paper_2002_05265_amd import inputs
from paper_2002_05265_amd.sim import Sim

pytestmark = pytest.mark.gpu

CENTRAL = {"CM", "CHM", "K"}
CASES = [(m, N) for m in inputs.MODEL_NAMES for N in ([4] if m in CENTRAL else [2, 3, 4])]


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def cells():
    n = 1000
    rng = np.random.default_rng(2002)
    f = inputs.random_cells(n * n, rng)  # [cells, 9]
    f = np.ascontiguousarray(f.T.reshape(9, n, n))
    rho = f.sum(axis=0)
    ux = (f[1] + f[5] + f[8] - f[3] - f[6] - f[7]) / rho
    uy = (f[2] + f[5] + f[6] - f[4] - f[7] - f[8]) / rho
    return f, rho, ux, uy


@pytest.mark.parametrize("name,N", CASES)
def test_random_cells(gpu, cells, name, N):
    f, rho, ux, uy = cells
    omega = np.array([1.93, 1.7, 1.2, 0.8, 1.45])
    sim = Sim(rho, ux, uy, prec="f64", eq_order=N, device=gpu)
    try:
        assert sim.fusion_depth(name) == 3  # one fused launch advances three steps on this grid
        for steps, bar in ((1, 1e-13), (3, 1e-12)):
            sim.set_state(f, 0)
            sim.step(name, omega, steps)
            got = sim.state().cpu().numpy()
            ref = oracle.step(f, inputs.MODEL_CODES[name], N, omega, steps)
            e = rel(got, ref)
            print(f"random cells {name} N={N} {steps} step(s): {e:.2e}", flush=True)
            assert e < bar, (name, N, steps, e)
    finally:
        sim.close()


def mode_amplitude(field, n):
    """Complex amplitude of the first Fourier mode along x, averaged over y."""
    x = np.arange(n)
    return np.mean(field @ np.exp(-2j * np.pi * x / n)) * 2.0 / n


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["BGK", "RM", "CM", "K", "RR"])
def test_shear_wave_viscosity(gpu, prec, name):
    n, nu, mach, steps, chunk = 64, 0.05, 0.1, 1500, 100
    rho, ux, uy = inputs.shear_wave_fields(n, mach)
    omega = inputs.rates(nu, "SRT")
    sim = Sim(rho, ux, uy, prec=prec, eq_order=4, device=gpu, ref_velocity=(mach * inputs.CS, 0.0))
    ts, amps = [], []
    for t in range(0, steps + 1, chunk):
        if t:
            sim.step(name, omega, chunk)
        if t >= 200:
            _, _, v, _ = sim.moments()
            ts.append(t)
            amps.append(abs(mode_amplitude(v.cpu().numpy(), n)))
    sim.close()
    k = 2 * np.pi / n
    ratio = -np.polyfit(ts, np.log(amps), 1)[0] / k ** 2 / nu
    print(f"shear wave {prec} {name}: nu_measured / nu = {ratio:.5f}", flush=True)
    assert abs(ratio - 1.0) < 5e-3, ratio


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["BGK", "CHM", "K", "RR"])
def test_sound_speed(gpu, prec, name):
    n, steps = 64, 360
    rho, ux, uy = inputs.sound_wave_fields(n)
    omega = inputs.rates(0.01, "SRT")
    sim = Sim(rho, ux, uy, prec=prec, eq_order=4, device=gpu)
    amps = []
    for _ in range(steps):
        sim.step(name, omega, 1)
        r, _, _, _ = sim.moments()
        amps.append(mode_amplitude(r.cpu().numpy() - 1.0, n).imag)
    sim.close()
    a = np.array(amps)
    # zero crossings of a standing wave cos(c k t): half-period spacing pi / (c k)
    z = [i + a[i] / (a[i] - a[i + 1]) for i in range(len(a) - 1) if a[i] * a[i + 1] < 0]
    c = np.pi / (np.mean(np.diff(z)) * 2 * np.pi / n)
    print(f"sound speed {prec} {name}: c sqrt(3) = {c * np.sqrt(3):.5f}", flush=True)
    assert abs(c * np.sqrt(3) - 1.0) < 5e-3, c
