"""Which readings of the cumulant (K) collision are admissible, and how each linearises.

The paper does not print its K collision; its Sections 4b, 4c and 5c report that K is the only
model with growing waves at rest, that SRT-K does not linearise like BGK, and that REG-K does
not recover SRT-RR as REG-CHM does.  This file settles, with the oracle's own Jacobians, what any
reading of K can give:

- A reading is admissible when the equilibrium is a fixed point at every (rho, u) and all rates
  equal to 1 return f^eq (every moment set to its equilibrium).  For such a transform T and its
  inverse, the SRT linearisation about f^eq is
      df* = DT^-1 [(1 - w) DT df + w dX^eq] = (1 - w) df + w df^eq,
  because DT df^eq = dX^eq when X^eq = T(f^eq): BGK's.  Under REG the fourth cumulant's first
  variation at f^eq, dk22 - cs^2 (dk20 + dk02) + cs^4 drho, is the central Hermite moment's, so
  REG-K linearises like REG-CHM.
- Checked over the readings the paper leaves open: cumulants of f / rho (rho-weighted products
  (k20 k02 + 2 k11^2) / rho) or unweighted products, the fourth cumulant's equilibrium 0 or its
  value at f^eq, and the fourth-order reconstruction from post- or pre-collision second-order
  cumulants.  Every admissible one has the Jacobian of CM (SRT) / CHM (REG), and the flow at rest is
  linearly stable.
- The readings that do change the linearisation break the fixed point or the all-rates-1 property,
  and are unstable at rest by 2-87 % per step: a run would blow up within a few hundred steps,
  against the paper's numerical finding (Section 5c) that SRT-K's stability domain is close to
  BGK's.  None of them is the paper's K either.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2002_05265_amd import inputs

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
CS2 = 1.0 / 3.0
PQ = [(p, q) for p in range(3) for q in range(3)]
RATES = [1.93, 1.41, 1.17, 0.83, 1.62]


def _relax(X, Xeq, w):
    """Appendix B relaxation with the five rates (trace / deviator split of the second order)."""
    wn, wb, w21, w12, w22 = w
    d = {pq: X[pq] - Xeq[pq] for pq in X}
    out = dict(X)
    s, dl = d[2, 0] + d[0, 2], d[2, 0] - d[0, 2]
    out[2, 0] = Xeq[2, 0] + 0.5 * ((1 - wb) * s + (1 - wn) * dl)
    out[0, 2] = Xeq[0, 2] + 0.5 * ((1 - wb) * s - (1 - wn) * dl)
    out[1, 1] = Xeq[1, 1] + (1 - wn) * d[1, 1]
    out[2, 1] = Xeq[2, 1] + (1 - w21) * d[2, 1]
    out[1, 2] = Xeq[1, 2] + (1 - w12) * d[1, 2]
    out[2, 2] = Xeq[2, 2] + (1 - w22) * d[2, 2]
    return out


def k_collide(f, w, weighted=True, eq22="feq", recon="post"):
    """One cumulant collision under a given reading.  Central moments come from the 9 x 9 matrix
    of the peculiar-velocity monomials, and the post-collision populations from solving it."""
    rho = f.sum()
    ux, uy = (CX * f).sum() / rho, (CY * f).sum() / rho
    T = np.array([(CX - ux) ** p * (CY - uy) ** q for p, q in PQ])
    k = dict(zip(PQ, T @ f))
    norm = rho if weighted else 1.0
    K = dict(k)
    K[2, 2] = k[2, 2] - (k[2, 0] * k[0, 2] + 2 * k[1, 1] ** 2) / norm
    Keq = {pq: 0.0 * rho for pq in PQ}
    Keq[0, 0], Keq[2, 0], Keq[0, 2] = rho, rho * CS2, rho * CS2
    Keq[2, 2] = 0.0 * rho if eq22 == "zero" else rho * CS2 * CS2 - (rho * CS2) ** 2 / norm
    Ks = _relax(K, Keq, w)
    low = Ks if recon == "post" else k
    ks = dict(Ks)
    ks[2, 2] = Ks[2, 2] + (low[2, 0] * low[0, 2] + 2 * low[1, 1] ** 2) / norm
    return np.linalg.solve(T, np.array([ks[pq] for pq in PQ]))


def jacobian(fn, f):
    """Complex-step Jacobian (Squire and Trapp): exact to rounding for a rational map."""
    h = 1e-30
    cols = [fn(f.astype(complex) + 1j * h * np.eye(9)[j]).imag / h for j in range(9)]
    return np.array(cols).T


def rest_growth(J, n=33):
    """max |eigenvalue| - 1 of M^D(k) over an n x n grid of k in [-pi, pi]^2."""
    ks = np.linspace(-math.pi, math.pi, n)
    return max(np.max(np.abs(oracle.lsa_eigenvalues(J, a, b))) for a in ks for b in ks) - 1.0


def _state(seed=1):
    rng = np.random.default_rng(seed)
    return oracle.feq_cell(4, 1.03, 0.11, -0.07) * (1 + 0.05 * rng.standard_normal(9))


READINGS = list(itertools.product([True, False], ["zero", "feq"], ["post", "pre"]))


def admissible(weighted, eq22, recon):
    f = _state()
    fe = oracle.feq_cell(4, 1.07, 0.1, 0.05)
    rho = f.sum()
    ones = k_collide(f, [1.0] * 5, weighted, eq22, recon)
    fixed = np.max(np.abs(k_collide(fe, RATES, weighted, eq22, recon) - fe)) < 1e-14
    to_eq = np.max(np.abs(ones - oracle.feq_cell(4, rho, (CX * f).sum() / rho, (CY * f).sum() / rho))) < 1e-14
    return fixed and to_eq


def test_textbook_reading_is_the_oracle_k():
    # pins this file's helper to the oracle (rho-weighted, equilibrium 0 = its f^eq value, post)
    for seed in range(4):
        f = _state(seed)
        for w in (RATES, [1.7] * 5, [1.2, 1.2, 1.0, 1.0, 1.0]):
            np.testing.assert_allclose(k_collide(f, w, True, "zero", "post"),
                                       oracle.collide_cell(oracle.K, 4, w, f), atol=2e-15)


@pytest.mark.parametrize("weighted,eq22,recon", READINGS)
def test_admissible_readings_linearise_like_cm_and_chm(weighted, eq22, recon):
    if not admissible(weighted, eq22, recon):
        pytest.skip("not admissible (checked in the next test)")
    for mach, phi in ((0.0, 0.0), (0.3, 0.4)):
        u = mach * math.sqrt(CS2)
        fe = oracle.feq_cell(4, 1.0, u * math.cos(phi), u * math.sin(phi))
        for preset, other in (("SRT", oracle.CM), ("REG", oracle.CHM)):
            w = inputs.rates(1e-6, preset)
            Jk = jacobian(lambda f: k_collide(f, w, weighted, eq22, recon), fe)
            Jo = oracle.collide_jacobian(other, 4, w, fe)[0]
            np.testing.assert_allclose(Jk, Jo, atol=1e-13)
            if mach == 0.0:
                assert rest_growth(Jk) < 1e-12


@pytest.mark.parametrize("weighted,eq22,recon", READINGS)
def test_readings_that_change_the_linearisation_are_inadmissible(weighted, eq22, recon):
    fe = oracle.feq_cell(4, 1.0, 0.0, 0.0)
    changed = False
    for preset, other in (("SRT", oracle.CM), ("REG", oracle.CHM)):
        w = inputs.rates(1e-6, preset)
        Jk = jacobian(lambda f: k_collide(f, w, weighted, eq22, recon), fe)
        if np.max(np.abs(Jk - oracle.collide_jacobian(other, 4, w, fe)[0])) > 1e-10:
            changed = True
            # unstable at rest by at least 2 % per step: blow-up within a few hundred steps
            assert rest_growth(Jk) > 0.02
    assert changed == (not admissible(weighted, eq22, recon))
