"""Pins of the oracle's discrete equilibrium against closed forms fixed by the paper.

- Section 2, eq. extendedFeq: the product (left-hand) form of the extended equilibrium,
  written out here independently of the oracle's raw-moment (right-hand) form.
- Section 2, matching conditions: the nine raw moments (p, q <= 2) of the extended
  equilibrium equal those of the Maxwellian, rho E[xi_x^p] E[xi_y^q] with xi ~ N(u, cs^2 I).
- At rest the equilibrium reduces to the D2Q9 weights 4/9, 1/9, 1/36 (T0 = cs^2 = 1/3).
- The second-order equilibrium (Hermite truncation reading) equals the textbook polynomial
  w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2].
"""
import numpy as np
import pytest

import oracle

CX, CY = oracle.CX.astype(float), oracle.CY.astype(float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
CS2 = 1.0 / 3.0

rng = np.random.default_rng(11)
STATES = [(1.0, 0.0, 0.0)] + [(float(r), float(u), float(v)) for r, u, v in
                              zip(rng.uniform(0.8, 1.2, 12), rng.uniform(-0.3, 0.3, 12),
                                  rng.uniform(-0.3, 0.3, 12))]


def raw_moment(f, p, q):
    return float(np.sum(CX ** p * CY ** q * f))


def gauss_moment(m, p):
    return {0: 1.0, 1: m, 2: m * m + CS2, 3: m ** 3 + 3 * m * CS2}[p]


@pytest.mark.parametrize("N", [2, 3, 4])
def test_rest_weights(N):
    for rho in (1.0, 0.7, 1.3):
        np.testing.assert_allclose(oracle.feq_cell(N, rho, 0.0, 0.0), rho * W, rtol=0, atol=1e-15)


@pytest.mark.parametrize("rho,ux,uy", STATES)
def test_product_form(rho, ux, uy):
    # eq. extendedFeq, left-hand forms with M^eq of the Maxwellian (M22 = M20 M02 / rho)
    M00, M10, M01 = rho, rho * ux, rho * uy
    M20, M02 = rho * (ux * ux + CS2), rho * (uy * uy + CS2)
    f = np.empty(9)
    for i in range(9):
        s, l = CX[i], CY[i]
        ax = (M00 - M20) if s == 0 else 0.5 * (s * M10 + M20)
        ay = (M00 - M02) if l == 0 else 0.5 * (l * M01 + M02)
        f[i] = ax * ay / rho
    np.testing.assert_allclose(oracle.feq_cell(4, rho, ux, uy), f, rtol=0, atol=2e-16)


@pytest.mark.parametrize("rho,ux,uy", STATES)
def test_matching_conditions(rho, ux, uy):
    fe4 = oracle.feq_cell(4, rho, ux, uy)
    fe3 = oracle.feq_cell(3, rho, ux, uy)
    fe2 = oracle.feq_cell(2, rho, ux, uy)
    for p in range(3):
        for q in range(3):
            mb = rho * gauss_moment(ux, p) * gauss_moment(uy, q)
            assert abs(raw_moment(fe4, p, q) - mb) < 1e-15, (p, q)
            if p + q <= 3:
                assert abs(raw_moment(fe3, p, q) - mb) < 1e-15, (p, q)
            if p + q <= 2:
                assert abs(raw_moment(fe2, p, q) - mb) < 1e-15, (p, q)
    # below order 4 the dropped Hermite terms show up exactly where expected
    if abs(ux * uy) > 1e-3:
        assert abs(raw_moment(fe3, 2, 2) - rho * gauss_moment(ux, 2) * gauss_moment(uy, 2)) > 1e-6
        assert abs(raw_moment(fe2, 2, 1) - rho * gauss_moment(ux, 2) * uy) > 1e-6
    # aliasing xi^3 = xi: the third-order raw moment M30 equals M10 on D2Q9 (Section 2)
    assert abs(raw_moment(fe4, 3, 0) - rho * ux) < 1e-15


@pytest.mark.parametrize("rho,ux,uy", STATES)
def test_second_order_textbook(rho, ux, uy):
    cu = CX * ux + CY * uy
    ref = W * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
    np.testing.assert_allclose(oracle.feq_cell(2, rho, ux, uy), ref, rtol=0, atol=2e-16)


def test_init_eq_grid_matches_cells():
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.9, 1.1, (5, 7))
    ux = rng.uniform(-0.1, 0.1, (5, 7))
    uy = rng.uniform(-0.1, 0.1, (5, 7))
    for N in (2, 3, 4):
        f = oracle.init_eq(N, rho, ux, uy)
        for y in range(5):
            for x in range(7):
                np.testing.assert_array_equal(f[:, y, x], oracle.feq_cell(N, rho[y, x], ux[y, x], uy[y, x]))
        r, u, v, tot = oracle.moments(f)
        np.testing.assert_allclose(r, rho, rtol=1e-15)
        np.testing.assert_allclose(u, ux, atol=1e-16)
        np.testing.assert_allclose(v, uy, atol=1e-16)
        assert abs(tot[0] - rho.sum()) < 1e-12
        assert abs(tot[3] - np.sum(0.5 * rho * (ux ** 2 + uy ** 2))) < 1e-14
        assert abs(tot[4] - np.mean(ux ** 2 + uy ** 2)) < 1e-16
