"""Pins of the oracle's eight collision models (Appendix B) against what the paper fixes.

Each test recomputes what it needs from the definitions with numpy (or sympy), never through
the oracle's own transform code:
  * conservation of mass and momentum (eq. RMcoll / eq. CHMcoll / eq. HMColl_Q9, the
    zeroth- and first-order moments are kept);
  * f = f^eq is a fixed point, and all rates equal to 1 give f* = f^eq;
  * relaxation in each model's own space: the moments of f* (recomputed here from their
    definitions) equal X^eq + (1 - omega)(X - X^eq) with the paper's (omega_nu, omega_3,
    omega_4) (eq. RMcoll, eq. CHMcoll, eq. HMColl_Q9 with eq. RRformulas_D2Q9); for K the
    textbook cumulants are obtained by differentiating the log moment generating function;
  * SRT: RM, HM, CM and CHM coincide with BGK, K and RR do not (Sections 4c and 5c);
  * REG: CHM coincides with SRT-RR; HM and RR coincide with PR (Sections 4c and 5c);
  * a closed form, derived from the cumulant definition, of the only difference between
    SRT-K and BGK (a change of the fourth-order central moment).
"""
import numpy as np
import pytest
import sympy as sp

import oracle
from paper_2002_05265_amd import inputs

CX, CY = oracle.CX.astype(float), oracle.CY.astype(float)
CS2 = 1.0 / 3.0
CELLS = inputs.random_cells(24, np.random.default_rng(7), spread=0.05, umax=0.15)
ALL = ["BGK", "RM", "HM", "CM", "CHM", "K", "PR", "RR"]
CENTRAL = {"CM", "CHM", "K"}


def herm(p, z):
    return [np.ones_like(z), z, z * z - CS2][p]


def macro(f):
    rho = f.sum()
    return rho, np.dot(CX, f) / rho, np.dot(CY, f) / rho


def moments(kind, f, ux=0.0, uy=0.0):
    X = np.zeros((3, 3))
    for p in range(3):
        for q in range(3):
            if kind == "raw":
                w = CX ** p * CY ** q
            elif kind == "hermite":
                w = herm(p, CX) * herm(q, CY)
            elif kind == "central":
                w = (CX - ux) ** p * (CY - uy) ** q
            else:
                w = herm(p, CX - ux) * herm(q, CY - uy)
            X[p, q] = np.dot(w, f)
    return X


def paper_relax(X, Xeq, wnu, w3, w4):
    """X* = (1 - omega) X + omega X^eq per moment (eq. RMcoll form)."""
    Y = X.copy()
    for (p, q), w in {(2, 0): wnu, (0, 2): wnu, (1, 1): wnu, (2, 1): w3, (1, 2): w3, (2, 2): w4}.items():
        Y[p, q] = (1 - w) * X[p, q] + w * Xeq[p, q]
    return Y


def paper_omega(wnu, w3, w4):
    return [wnu, wnu, w3, w3, w4]


def collide(name, N, omega, f):
    return oracle.collide_cell(oracle.MODELS[name], N, omega, f)


def orders(name):
    return [4] if name in CENTRAL else [2, 3, 4]


@pytest.mark.parametrize("name", ALL)
def test_conservation(name):
    for N in orders(name):
        for f in CELLS:
            for omega in (paper_omega(1.7, 1.2, 0.8), [1.99, 0.6, 1.3, 0.4, 1.8]):
                g = collide(name, N, omega, f)
                assert abs(g.sum() - f.sum()) < 1e-15
                assert abs(np.dot(CX, g) - np.dot(CX, f)) < 1e-15
                assert abs(np.dot(CY, g) - np.dot(CY, f)) < 1e-15


@pytest.mark.parametrize("name", ALL)
def test_fixed_point_and_unit_rates(name):
    for N in orders(name):
        for f in CELLS[:8]:
            rho, ux, uy = macro(f)
            fe = oracle.feq_cell(N, rho, ux, uy)
            g = collide(name, N, [1.93, 1.4, 0.7, 1.1, 1.6], fe)
            np.testing.assert_allclose(g, fe, rtol=0, atol=1e-15)
            g1 = collide(name, N, [1.0] * 5, f)
            np.testing.assert_allclose(g1, fe, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name,kind", [("RM", "raw"), ("HM", "hermite"), ("CM", "central"),
                                       ("CHM", "central_hermite")])
def test_relaxation_in_own_space(name, kind):
    wnu, w3, w4 = 1.87, 1.31, 0.63
    for N in orders(name):
        for f in CELLS:
            rho, ux, uy = macro(f)
            fe = oracle.feq_cell(N, rho, ux, uy)
            g = collide(name, N, paper_omega(wnu, w3, w4), f)
            X, Xeq, Xs = (moments(kind, h, ux, uy) for h in (f, fe, g))
            ref = paper_relax(X, Xeq, wnu, w3, w4)
            np.testing.assert_allclose(Xs, ref, rtol=0, atol=2e-15)


def test_hermite_equilibrium_in_central_spaces():
    # eq. CHMcoll: the central Hermite moments of f^eq (order 4) vanish except the zeroth
    for f in CELLS[:6]:
        rho, ux, uy = macro(f)
        At = moments("central_hermite", oracle.feq_cell(4, rho, ux, uy), ux, uy)
        ref = np.zeros((3, 3))
        ref[0, 0] = rho
        np.testing.assert_allclose(At, ref, atol=1e-15)


def test_bulk_rate_relaxes_trace_only():
    # with omega_b != omega_nu the trace of the second-order non-equilibrium block decays
    # with omega_b and the deviator with omega_nu, in every moment-space model
    wnu, wb = 1.9, 1.2
    for name in ["RM", "HM", "CM", "CHM", "K", "RR", "PR"]:
        for f in CELLS[:6]:
            rho, ux, uy = macro(f)
            fe = oracle.feq_cell(4, rho, ux, uy)
            g = collide(name, 4, [wnu, wb, 1.0, 1.0, 1.0], f)
            d, ds = moments("raw", f) - moments("raw", fe), moments("raw", g) - moments("raw", fe)
            assert abs((ds[2, 0] + ds[0, 2]) - (1 - wb) * (d[2, 0] + d[0, 2])) < 1e-15
            assert abs((ds[2, 0] - ds[0, 2]) - (1 - wnu) * (d[2, 0] - d[0, 2])) < 1e-15
            assert abs(ds[1, 1] - (1 - wnu) * d[1, 1]) < 1e-15


def test_recursive_regularized_moments():
    # eq. HMColl_Q9 with eq. RRformulas_D2Q9: A*_pq = A^eq_pq + (1 - omega) A^neq_pq with the
    # recursive third and fourth order non-equilibrium moments
    wnu, w3, w4 = 1.95, 1.4, 0.7
    for N in (2, 3, 4):
        for f in CELLS:
            rho, ux, uy = macro(f)
            A = moments("hermite", f)
            Aeq = moments("hermite", oracle.feq_cell(N, rho, ux, uy))
            As = moments("hermite", collide("RR", N, paper_omega(wnu, w3, w4), f))
            n20, n02, n11 = A[2, 0] - Aeq[2, 0], A[0, 2] - Aeq[0, 2], A[1, 1] - Aeq[1, 1]
            n21 = uy * n20 + 2 * ux * n11
            n12 = ux * n02 + 2 * uy * n11
            n22 = uy * uy * n20 + ux * ux * n02 + 4 * ux * uy * n11
            ref = {(2, 0): Aeq[2, 0] + (1 - wnu) * n20, (0, 2): Aeq[0, 2] + (1 - wnu) * n02,
                   (1, 1): Aeq[1, 1] + (1 - wnu) * n11, (2, 1): Aeq[2, 1] + (1 - w3) * n21,
                   (1, 2): Aeq[1, 2] + (1 - w3) * n12, (2, 2): Aeq[2, 2] + (1 - w4) * n22}
            for (p, q), v in ref.items():
                assert abs(As[p, q] - v) < 2e-15, (N, p, q)


def test_pr_equilibrates_high_orders():
    for N in (2, 3, 4):
        for f in CELLS:
            rho, ux, uy = macro(f)
            Aeq = moments("hermite", oracle.feq_cell(N, rho, ux, uy))
            A = moments("hermite", f)
            As = moments("hermite", collide("PR", N, [1.8, 1.8, 0.3, 0.4, 0.5], f))
            for p, q in [(2, 1), (1, 2), (2, 2)]:
                assert abs(As[p, q] - Aeq[p, q]) < 2e-15
            assert abs(As[1, 1] - (Aeq[1, 1] + (1 - 1.8) * (A[1, 1] - Aeq[1, 1]))) < 2e-15


def cumulants_sympy(f):
    """kappa_pq of the distribution f / rho over the lattice velocities, from the log moment
    generating function log sum_i (f_i / rho) exp(s xi_x + t xi_y)."""
    s, t = sp.symbols("s t")
    rho = f.sum()
    mgf = sum(sp.Float(fi / rho, 30) * sp.exp(s * int(a) + t * int(b)) for fi, a, b in zip(f, CX, CY))
    K = sp.log(mgf)
    out = {}
    for p, q in [(2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]:
        d = sp.diff(K, s, p, t, q) if p and q else (sp.diff(K, s, p) if p else sp.diff(K, t, q))
        out[(p, q)] = float(d.subs({s: 0, t: 0}).evalf(25))
    return out


def test_cumulant_relaxation_textbook():
    wnu, w3, w4 = 1.85, 1.25, 0.55
    for f in CELLS[:5]:
        rho, ux, uy = macro(f)
        k0 = cumulants_sympy(f)
        k1 = cumulants_sympy(collide("K", 4, paper_omega(wnu, w3, w4), f))
        eq = {(2, 0): CS2, (0, 2): CS2, (1, 1): 0.0, (2, 1): 0.0, (1, 2): 0.0, (2, 2): 0.0}
        rate = {(2, 0): wnu, (0, 2): wnu, (1, 1): wnu, (2, 1): w3, (1, 2): w3, (2, 2): w4}
        for pq in eq:
            ref = eq[pq] + (1 - rate[pq]) * (k0[pq] - eq[pq])
            assert abs(k1[pq] - ref) < 5e-15, pq


@pytest.mark.parametrize("name", ["RM", "HM", "CM", "CHM"])
def test_srt_moment_models_equal_bgk(name):
    for N in orders(name):
        for f in CELLS:
            for w in (1.9, 1.999988, 0.8):
                np.testing.assert_allclose(collide(name, N, [w] * 5, f), collide("BGK", N, [w] * 5, f),
                                           rtol=0, atol=2e-16 * 8)


def test_srt_k_differs_from_bgk_by_closed_form():
    # Under SRT with rate w, K and BGK differ only in the fourth-order central moment:
    # dk22 = -w (1 - w) rho (a b + 2 c^2), a = k20/rho - cs2, b = k02/rho - cs2, c = k11/rho,
    # i.e. in populations dk22 * (1, -1/2 x4, 1/4 x4) (eq. Q9postCollVDF_RM with M22 only).
    shape = np.array([1.0, -0.5, -0.5, -0.5, -0.5, 0.25, 0.25, 0.25, 0.25])
    for f in CELLS:
        rho, ux, uy = macro(f)
        k = moments("central", f, ux, uy)
        a, b, c = k[2, 0] / rho - CS2, k[0, 2] / rho - CS2, k[1, 1] / rho
        for w in (1.9, 1.5, 0.7):
            dk22 = -w * (1 - w) * rho * (a * b + 2 * c * c)
            diff = collide("K", 4, [w] * 5, f) - collide("BGK", 4, [w] * 5, f)
            np.testing.assert_allclose(diff, dk22 * shape, rtol=0, atol=2e-16 * 8)
            assert np.max(np.abs(diff)) > 1e-9  # K is not BGK (Sections 4c and 5c)


def test_srt_rr_differs_from_bgk():
    for f in CELLS[:6]:
        assert np.max(np.abs(collide("RR", 4, [1.9] * 5, f) - collide("BGK", 4, [1.9] * 5, f))) > 1e-6


@pytest.mark.parametrize("N", [2, 3, 4])
def test_reg_hm_rr_pr_coincide(N):
    for f in CELLS:
        for w in (1.9, 1.999988):
            reg = [w, w, 1.0, 1.0, 1.0]
            pr = collide("PR", N, reg, f)
            np.testing.assert_allclose(collide("HM", N, reg, f), pr, rtol=0, atol=4e-16)
            np.testing.assert_allclose(collide("RR", N, reg, f), pr, rtol=0, atol=4e-16)


def test_reg_chm_equals_srt_rr():
    for f in CELLS:
        for w in (1.9, 1.999988, 1.3):
            np.testing.assert_allclose(collide("CHM", 4, [w, w, 1.0, 1.0, 1.0], f),
                                       collide("RR", 4, [w] * 5, f), rtol=0, atol=4e-16)


def test_unsupported_orders_rejected():
    f = CELLS[0]
    for name in CENTRAL:
        for N in (2, 3):
            with pytest.raises(ValueError):
                collide(name, N, [1.9] * 5, f)
