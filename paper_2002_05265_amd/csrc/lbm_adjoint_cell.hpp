// Hand-written reverse mode of the per-cell collision in lbm_cell.hpp.
//
// Given mu = dL/dh* (the adjoint of the post-collision populations), collide_adjoint returns
// hb = dL/dh = J_C(h)^T mu and the adjoints of the relaxation coefficients.  The forward pass
// is recomputed step by step (the "tape" lives in registers) and every statement of
// lbm_cell.hpp is then reversed in the opposite order:
//
//   F1 drho, jx, jy = sums of h            R1 hb_i += drho_b + cx_i jx_b + cy_i jy_b
//   F2 rho, du, u                          R2 quotient rule, u = U + du
//   F3 E = hermite_eq(drho, u, du)         R3 eq_adjoint (telescoped monomials)
//   F4 d = A(h) - E                        R4 neq_adjoint (linear in h, minus E)
//   F5 n = relax_model(d, u, rho, coef)    R5 per-model reverse
//   F6 h* = P(drho, jx, jy, E + n)         R6 pop_adjoint (transpose of a linear map)
//
// Coefficient adjoints cb = (cpp, cpm, c11, c21, c12, c22, om) map to the rates by
// omega_b(cpp, cpm, c11, om): d/domega_nu = -cpp/2 + cpm/2 - c11 + om,
// d/domega_b = -cpp/2 - cpm/2, d/domega_21 = -c21, d/domega_12 = -c12, d/domega_22 = -c22.
#pragma once

#include "lbm_cell.hpp"

namespace lbm {

template <typename R> struct MacroBar {
    R drho, rho, jx, jy, ux, uy, dux, duy;
};

template <typename R>
__device__ __forceinline__ void zero(MacroBar<R>& b) {
    b.drho = b.rho = b.jx = b.jy = b.ux = b.uy = b.dux = b.duy = R(0);
}

// R6: transpose of hermite_to_pop.  Outputs the adjoints of drho, jx, jy and of the six
// post-collision Hermite differences a20 .. a22.
template <typename R>
__device__ __forceinline__ void pop_adjoint(const R (&mu)[9], MacroBar<R>& mb, R (&ab)[6]) {
    using L = Lat<R>;
    const R r0b = mu[0];
    const R r1b = (mu[1] + mu[3]) + (mu[2] + mu[4]);
    const R r5b = (mu[5] + mu[6]) + (mu[7] + mu[8]);
    const R hxb = mu[1] + mu[3], pxb = mu[1] - mu[3];
    const R hyb = mu[2] + mu[4], pyb = mu[2] - mu[4];
    const R qb = r5b;
    const R s11b = (mu[5] + mu[7]) - (mu[6] + mu[8]);
    const R s12b = (mu[5] + mu[8]) - (mu[6] + mu[7]);
    const R s21b = (mu[5] + mu[6]) - (mu[7] + mu[8]);
    const R M22b = mu[0] - R(0.5) * (hxb + hyb) + R(0.25) * qb;
    const R M20b = R(0.5) * hxb - mu[0];
    const R M02b = R(0.5) * hyb - mu[0];
    const R M12b = R(0.25) * s12b - R(0.5) * pxb;
    const R M21b = R(0.25) * s21b - R(0.5) * pyb;
    const R M11b = R(0.25) * s11b;
    mb.jx += R(0.5) * pxb + L::cs2 * M12b;
    mb.jy += R(0.5) * pyb + L::cs2 * M21b;
    mb.drho += L::w0 * r0b + L::w1 * r1b + L::w5 * r5b;
    ab[0] = M20b + L::cs2 * M22b;  // a20
    ab[1] = M02b + L::cs2 * M22b;  // a02
    ab[2] = M11b;                  // a11
    ab[3] = M21b;                  // a21
    ab[4] = M12b;                  // a12
    ab[5] = M22b;                  // a22
}

// R3: reverse of hermite_eq.  eb = adjoints of (e20, e02, e11, e21, e12, e22).
template <typename R>
__device__ __forceinline__ void eq_adjoint(const Macro<R>& m, const Ref<R>& r, int N, const R (&eb)[6],
                                           MacroBar<R>& mb) {
    const R a = m.ux, b = m.uy, A = r.ux, da = m.dux, db = m.duy, dr = m.drho, rs = r.rho;
    const R a2 = a * a, b2 = b * b;
    const R D20 = da * (a + A);
    const R D02 = db * (b + r.uy);
    const R e20b = eb[0], e02b = eb[1], e11b = eb[2];
    const R e21b = N >= 3 ? eb[3] : R(0), e12b = N >= 3 ? eb[4] : R(0), e22b = N >= 4 ? eb[5] : R(0);
    // direct drho terms
    mb.drho += e20b * a2 + e02b * b2 + e11b * (a * b) + e21b * (a2 * b) + e12b * (a * b2) + e22b * (a2 * b2);
    R ab = dr * (R(2) * a * e20b + b * e11b + R(2) * a * b * e21b + b2 * e12b + R(2) * a * b2 * e22b);
    R bb = dr * (R(2) * b * e02b + a * e11b + a2 * e21b + R(2) * a * b * e12b + R(2) * a2 * b * e22b);
    // reference-difference terms
    const R D22b = rs * e22b, D21b = rs * e21b, D12b = rs * e12b, D11b = rs * e11b;
    const R D20b = rs * e20b + b * D21b + b2 * D22b;
    const R D02b = rs * e02b + A * D12b + (A * A) * D22b;
    R dab = R(0), dbb = R(0);
    bb += D20 * D21b;                 // D21 = D20 b + A^2 db
    dbb += (A * A) * D21b;
    dab += b2 * D12b;                 // D12 = da b^2 + A D02
    bb += R(2) * da * b * D12b;
    bb += R(2) * b * D20 * D22b;      // D22 = D20 b^2 + A^2 D02
    dab += b * D11b;                  // D11 = da b + A db
    bb += da * D11b;
    dbb += A * D11b;
    dab += (a + A) * D20b;            // D20 = da (a + A)
    ab += da * D20b;
    dbb += (b + r.uy) * D02b;         // D02 = db (b + B)
    bb += db * D02b;
    mb.ux += ab;
    mb.uy += bb;
    mb.dux += dab;
    mb.duy += dbb;
}

// R4: reverse of hermite_neq (d = A(h) - E).  Adds to hb, mb and eb (eb -= db).
template <typename R>
__device__ __forceinline__ void neq_adjoint(const R (&db)[6], R (&hb)[9], MacroBar<R>& mb, R (&eb)[6]) {
    using L = Lat<R>;
    for (int k = 0; k < 6; ++k) eb[k] -= db[k];
    const R a22b = db[5];
    const R a20b = db[0] - L::cs2 * a22b;
    const R a02b = db[1] - L::cs2 * a22b;
    mb.drho -= L::cs2 * (a20b + a02b) + L::cs4 * a22b;
    mb.jy -= L::cs2 * db[3];
    mb.jx -= L::cs2 * db[4];
    const R m20b = a20b, m02b = a02b, m11b = db[2], m21b = db[3], m12b = db[4];
    const R diagb = a22b + m20b + m02b;
    hb[1] += m20b;
    hb[3] += m20b;
    hb[2] += m02b;
    hb[4] += m02b;
    hb[5] += diagb + m11b + m21b + m12b;
    hb[6] += diagb - m11b + m21b - m12b;
    hb[7] += diagb + m11b - m21b - m12b;
    hb[8] += diagb - m11b - m21b + m12b;
}

// R2 + R1: reverse of macro_of, adding to hb.
template <typename R>
__device__ __forceinline__ void macro_adjoint(const Macro<R>& m, const Ref<R>& r, MacroBar<R>& mb,
                                              R (&hb)[9]) {
    mb.dux += mb.ux;  // u = U + du
    mb.duy += mb.uy;
    const R inv = m.inv_rho;
    // du = (j - drho U) / rho
    mb.jx += mb.dux * inv;
    mb.jy += mb.duy * inv;
    mb.drho -= (r.ux * mb.dux + r.uy * mb.duy) * inv;
    mb.rho -= (m.dux * mb.dux + m.duy * mb.duy) * inv;
    mb.drho += mb.rho;  // rho = rho_s + drho
    hb[0] += mb.drho;
    hb[1] += mb.drho + mb.jx;
    hb[2] += mb.drho + mb.jy;
    hb[3] += mb.drho - mb.jx;
    hb[4] += mb.drho - mb.jy;
    hb[5] += mb.drho + mb.jx + mb.jy;
    hb[6] += mb.drho - mb.jx + mb.jy;
    hb[7] += mb.drho - mb.jx - mb.jy;
    hb[8] += mb.drho + mb.jx - mb.jy;
}

// Reverse of the whole collision of one cell.  cb: adjoints of (cpp, cpm, c11, c21, c12, c22,
// om), accumulated (+=).
template <int MODEL, typename R>
__device__ __forceinline__ void collide_adjoint(const R (&h)[9], const Macro<R>& m, const Ref<R>& ref,
                                                const Coef<R>& c, int N, const R (&mu)[9], R (&hb)[9],
                                                R (&cb)[7]) {
    using L = Lat<R>;
    MacroBar<R> mb;
    zero(mb);
    R eb[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int i = 0; i < 9; ++i) hb[i] = R(0);
    if constexpr (MODEL == kStreamOnly) {
#pragma unroll
        for (int i = 0; i < 9; ++i) hb[i] = mu[i];
        return;
    } else {
        const Eq<R> e = hermite_eq(m, ref, N);
        if constexpr (MODEL == kBGK) {
            // h* = h - om (h - heq), heq = P(drho, jx, jy, E)
            R heq[9];
            hermite_to_pop(m, e.e20, e.e02, e.e11, e.e21, e.e12, e.e22, heq);
            R heqb[9];
            R omb = R(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                hb[i] = (R(1) - c.om) * mu[i];
                heqb[i] = c.om * mu[i];
                omb += mu[i] * (heq[i] - h[i]);
            }
            cb[6] += omb;
            R ab[6];
            pop_adjoint(heqb, mb, ab);
            for (int k = 0; k < 6; ++k) eb[k] += ab[k];
        } else {
            const Neq<R> d = hermite_neq(h, m, e);
            // forward of the relaxation (the tape)
            const R n20 = c.cpp * d.d20 + c.cpm * d.d02;
            const R n02 = c.cpm * d.d20 + c.cpp * d.d02;
            const R n11 = c.c11 * d.d11;
            // R6: post-collision populations
            R ab[6];
            pop_adjoint(mu, mb, ab);
            // A* = E + n
            for (int k = 0; k < 6; ++k) eb[k] += ab[k];
            R n20b = ab[0], n02b = ab[1], n11b = ab[2];
            const R n21b = ab[3], n12b = ab[4], n22b = ab[5];
            R d20b = R(0), d02b = R(0), d11b = R(0), d21b = R(0), d12b = R(0), d22b = R(0);
            const R ux = m.ux, uy = m.uy;
            if constexpr (MODEL == kHM) {
                d21b += c.c21 * n21b; cb[3] += d.d21 * n21b;
                d12b += c.c12 * n12b; cb[4] += d.d12 * n12b;
                d22b += c.c22 * n22b; cb[5] += d.d22 * n22b;
            } else if constexpr (MODEL == kPR) {
                // n21 = n12 = n22 = 0
            } else if constexpr (MODEL == kRM) {
                d21b += c.c21 * n21b; cb[3] += d.d21 * n21b;
                d12b += c.c12 * n12b; cb[4] += d.d12 * n12b;
                // n22 = c22 (d22 + cs2 (d20 + d02)) - cs2 (n20 + n02)
                const R x22 = d.d22 + L::cs2 * (d.d20 + d.d02);
                cb[5] += x22 * n22b;
                d22b += c.c22 * n22b;
                d20b += c.c22 * L::cs2 * n22b;
                d02b += c.c22 * L::cs2 * n22b;
                n20b -= L::cs2 * n22b;
                n02b -= L::cs2 * n22b;
            } else if constexpr (MODEL == kRR) {
                const R r21 = uy * d.d20 + R(2) * ux * d.d11;
                const R r12 = ux * d.d02 + R(2) * uy * d.d11;
                const R r22 = uy * uy * d.d20 + ux * ux * d.d02 + R(4) * ux * uy * d.d11;
                cb[3] += r21 * n21b; cb[4] += r12 * n12b; cb[5] += r22 * n22b;
                const R r21b = c.c21 * n21b, r12b = c.c12 * n12b, r22b = c.c22 * n22b;
                d20b += uy * r21b + uy * uy * r22b;
                d02b += ux * r12b + ux * ux * r22b;
                d11b += R(2) * ux * r21b + R(2) * uy * r12b + R(4) * ux * uy * r22b;
                mb.uy += d.d20 * r21b + R(2) * d.d11 * r12b + (R(2) * uy * d.d20 + R(4) * ux * d.d11) * r22b;
                mb.ux += R(2) * d.d11 * r21b + d.d02 * r12b + (R(2) * ux * d.d02 + R(4) * uy * d.d11) * r22b;
            } else {  // kCM, kCHM, kK
                const R t21 = d.d21 - uy * d.d20 - R(2) * ux * d.d11;
                const R t12 = d.d12 - ux * d.d02 - R(2) * uy * d.d11;
                const R t22 = d.d22 - R(2) * (uy * d.d21 + ux * d.d12) + uy * uy * d.d20 +
                              ux * ux * d.d02 + R(4) * ux * uy * d.d11;
                const R s21 = c.c21 * t21;
                const R s12 = c.c12 * t12;
                // n21 = s21 + uy n20 + 2 ux n11 ; n12 = s12 + ux n02 + 2 uy n11
                // n22 = s22 + 2 (uy s21 + ux s12) + uy^2 n20 + ux^2 n02 + 4 ux uy n11
                const R s22b = n22b;
                const R s21b = n21b + R(2) * uy * n22b;
                const R s12b = n12b + R(2) * ux * n22b;
                n20b += uy * n21b + uy * uy * n22b;
                n02b += ux * n12b + ux * ux * n22b;
                n11b += R(2) * ux * n21b + R(2) * uy * n12b + R(4) * ux * uy * n22b;
                mb.uy += n20 * n21b + R(2) * n11 * n12b + (R(2) * s21 + R(2) * uy * n20 + R(4) * ux * n11) * n22b;
                mb.ux += R(2) * n11 * n21b + n02 * n12b + (R(2) * s12 + R(2) * ux * n02 + R(4) * uy * n11) * n22b;
                R t22b = R(0);
                if constexpr (MODEL == kCHM) {
                    cb[5] += t22 * s22b;
                    t22b += c.c22 * s22b;
                } else if constexpr (MODEL == kCM) {
                    const R x22 = t22 + L::cs2 * (d.d20 + d.d02);
                    cb[5] += x22 * s22b;
                    t22b += c.c22 * s22b;
                    d20b += c.c22 * L::cs2 * s22b;
                    d02b += c.c22 * L::cs2 * s22b;
                    n20b -= L::cs2 * s22b;
                    n02b -= L::cs2 * s22b;
                } else {  // kK
                    const R inv = m.inv_rho;
                    const R P = d.d20 * d.d02 + R(2) * d.d11 * d.d11;
                    const R Q = n20 * n02 + R(2) * n11 * n11;
                    cb[5] += (t22 - P * inv) * s22b;
                    t22b += c.c22 * s22b;
                    const R Pb = -c.c22 * inv * s22b;
                    const R Qb = inv * s22b;
                    const R invb = (Q - c.c22 * P) * s22b;
                    d20b += Pb * d.d02;
                    d02b += Pb * d.d20;
                    d11b += R(4) * Pb * d.d11;
                    n20b += Qb * n02;
                    n02b += Qb * n20;
                    n11b += R(4) * Qb * n11;
                    mb.rho -= invb * inv * inv;
                }
                const R t21b = c.c21 * s21b;
                const R t12b = c.c12 * s12b;
                cb[3] += t21 * s21b;
                cb[4] += t12 * s12b;
                // t22
                d22b += t22b;
                d21b -= R(2) * uy * t22b;
                d12b -= R(2) * ux * t22b;
                d20b += uy * uy * t22b;
                d02b += ux * ux * t22b;
                d11b += R(4) * ux * uy * t22b;
                mb.uy += (R(2) * uy * d.d20 - R(2) * d.d21 + R(4) * ux * d.d11) * t22b;
                mb.ux += (R(2) * ux * d.d02 - R(2) * d.d12 + R(4) * uy * d.d11) * t22b;
                // t21, t12
                d21b += t21b;
                d20b -= uy * t21b;
                d11b -= R(2) * ux * t21b;
                mb.uy -= d.d20 * t21b;
                mb.ux -= R(2) * d.d11 * t21b;
                d12b += t12b;
                d02b -= ux * t12b;
                d11b -= R(2) * uy * t12b;
                mb.ux -= d.d02 * t12b;
                mb.uy -= R(2) * d.d11 * t12b;
            }
            // second-order block, common to every moment space
            d20b += c.cpp * n20b + c.cpm * n02b;
            d02b += c.cpm * n20b + c.cpp * n02b;
            d11b += c.c11 * n11b;
            cb[0] += n20b * d.d20 + n02b * d.d02;
            cb[1] += n20b * d.d02 + n02b * d.d20;
            cb[2] += n11b * d.d11;
            const R dbv[6] = {d20b, d02b, d11b, d21b, d12b, d22b};
            neq_adjoint(dbv, hb, mb, eb);
        }
        eq_adjoint(m, ref, N, eb, mb);
        macro_adjoint(m, ref, mb, hb);
    }
}

// Adjoints of the five rates from the coefficient adjoints.
template <typename R>
__device__ __forceinline__ void omega_adjoint(const R (&cb)[7], double (&wb)[5]) {
    wb[0] = -0.5 * (double)cb[0] + 0.5 * (double)cb[1] - (double)cb[2] + (double)cb[6];
    wb[1] = -0.5 * (double)cb[0] - 0.5 * (double)cb[1];
    wb[2] = -(double)cb[3];
    wb[3] = -(double)cb[4];
    wb[4] = -(double)cb[5];
}

}  // namespace lbm
