// Per-cell D2Q9 collision for gfx950: moment transform -> relax -> back-transform, in registers.
//
// Every model of Appendix B (BGK, RM, HM, CM, CHM, K, PR, RR) is written here in one common
// "deviation" form so that the same code runs in FP64 and in FP32 on shifted populations:
//
//   stored value   h_i   = f_i - f^ref_i,  f^ref = f^eq_N(rho_s, U)   (a fixed reference state;
//                                           rho_s = 0, U = 0 for plain FP64 storage)
//   density        rho   = rho_s + drho,   drho = sum_i h_i
//   velocity       u     = U + du,         du = (sum_i xi_i h_i - drho U) / rho
//   every equilibrium moment enters as its difference to the reference, built from drho and du,
//   so each quantity carried through the transform is O(du), O(drho) or O(f^neq), never O(rho).
//
// Map used by every model (the pipeline of Appendix B):
//   1. h -> raw moments (eq. RMcoll definition) -> Hermite non-equilibrium d_pq = A_pq - A^eq_pq
//   2. relax d in the model's own space (RM: raw, HM/PR: Hermite, RR: recursive Hermite
//      (eq. RRformulas_D2Q9), CHM/CM/K: central (Hermite) moments obtained by the binomial shift
//      by -u of d, whose inverse is eq. CHM2HM_Q9)
//   3. A* = A^eq + d*  ->  raw moments (eq. HM2RM_Q9)  ->  populations (eq. Q9postCollVDF_RM)
//
// Relaxation vector (omega_nu, omega_b, omega_21, omega_12, omega_22): deviatoric and trace
// parts of the second-order block, then the two third-order and the fourth-order moment.
// The paper's (omega_nu, omega_3, omega_4) is omega_b = omega_nu, omega_21 = omega_12 = omega_3,
// omega_22 = omega_4 (eq. RMcoll, Section 4c).
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

enum Model : int {
    kBGK = 0, kRM = 1, kHM = 2, kCM = 3, kCHM = 4, kK = 5, kPR = 6, kRR = 7, kStreamOnly = 99
};
enum Prec : int { kF64 = 0, kF32 = 1, kF16 = 2 };

// Lattice constant c_s^2 = 1/3 and rest weights 4/9, 1/9, 1/36.
template <typename R> struct Lat {
    static constexpr R cs2 = R(1.0 / 3.0);
    static constexpr R cs4 = R(1.0 / 9.0);
    static constexpr R w0 = R(4.0 / 9.0);
    static constexpr R w1 = R(1.0 / 9.0);
    static constexpr R w5 = R(1.0 / 36.0);
};

// Velocity components, index order (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).
__host__ __device__ constexpr int cx(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0;
}
__host__ __device__ constexpr double rest_weight(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

// Relaxation coefficients in the form used by the kernels: (1 - omega) factors, with the
// second-order diagonal pair written as d20* = cpp d20 + cpm d02, d02* = cpm d20 + cpp d02.
template <typename R> struct Coef {
    R cpp, cpm, c11, c21, c12, c22, om;  // om = omega_nu (BGK)
};

template <typename R>
__host__ __device__ inline Coef<R> make_coef(const double w[5]) {
    const double a = 0.5 * (1.0 - w[1]);  // trace
    const double b = 0.5 * (1.0 - w[0]);  // deviator
    Coef<R> c;
    c.cpp = R(a + b);
    c.cpm = R(a - b);
    c.c11 = R(1.0 - w[0]);
    c.c21 = R(1.0 - w[2]);
    c.c12 = R(1.0 - w[3]);
    c.c22 = R(1.0 - w[4]);
    c.om = R(w[0]);
    return c;
}

// Reference state of the stored deviations (density rho_s, velocity U).
template <typename R> struct Ref {
    R rho, ux, uy;
};

// Conserved quantities of a cell: drho = rho - rho_s, (jx, jy) = rho u - rho_s U (the momentum
// of the stored deviations), u and du = u - U.
template <typename R> struct Macro {
    R drho, rho, jx, jy, ux, uy, dux, duy;
    R inv_rho;  // 1 / rho
};

// Hermite equilibrium moments of order N (A^eq_pq = rho ux^p uy^q, zero above order N), as
// differences to those of the reference: E_pq = A^eq_pq(rho, u) - A^eq_pq(rho_s, U)
//   = drho u^p v^q + rho_s (u^p v^q - U^p V^q),
// the monomial differences telescoped through du so that nothing of order one cancels.
template <typename R> struct Eq {
    R e20, e02, e11, e21, e12, e22;
};

template <typename R>
__host__ __device__ __forceinline__ Eq<R> hermite_eq(const Macro<R>& m, const Ref<R>& r, int N) {
    const R a = m.ux, b = m.uy, A = r.ux, da = m.dux, db = m.duy;
    const R a2 = a * a, b2 = b * b;
    const R D20 = da * (a + A);          // a^2 - A^2
    const R D02 = db * (b + r.uy);       // b^2 - B^2
    const R D11 = da * b + A * db;       // a b - A B
    Eq<R> e;
    e.e20 = m.drho * a2 + r.rho * D20;
    e.e02 = m.drho * b2 + r.rho * D02;
    e.e11 = m.drho * (a * b) + r.rho * D11;
    if (N >= 3) {
        const R D21 = D20 * b + (A * A) * db;  // a^2 b - A^2 B
        const R D12 = da * b2 + A * D02;       // a b^2 - A B^2
        e.e21 = m.drho * (a2 * b) + r.rho * D21;
        e.e12 = m.drho * (a * b2) + r.rho * D12;
    } else {
        e.e21 = R(0);
        e.e12 = R(0);
    }
    if (N >= 4) {
        const R D22 = D20 * b2 + (A * A) * D02;  // a^2 b^2 - A^2 B^2
        e.e22 = m.drho * (a2 * b2) + r.rho * D22;
    } else {
        e.e22 = R(0);
    }
    return e;
}

// Fused multiply-add, rounded once: written out where a product feeds a sum in another
// statement, so that every kernel (and the host) computes it the same way.
template <typename R>
__host__ __device__ __forceinline__ R fmadd(R a, R b, R c) {
    if constexpr (sizeof(R) == 4)
        return fmaf(a, b, c);
    else
        return fma(a, b, c);
}

// Post-collision Hermite moments minus the reference's (equilibrium difference + relaxed
// non-equilibrium part) -> raw-moment differences (eq. HM2RM_Q9, which is linear) -> stored
// deviations (eq. Q9postCollVDF_RM; the density difference contributes drho w_i).  The pairs of
// opposite populations share their sums and differences.
template <typename R>
__host__ __device__ __forceinline__ void hermite_to_pop(const Macro<R>& m, R a20, R a02, R a11, R a21,
                                               R a12, R a22, R (&h)[9]) {
    using L = Lat<R>;
    const R tr = a20 + a02;
    const R M21 = a21 + L::cs2 * m.jy;
    const R M12 = a12 + L::cs2 * m.jx;
    const R M22 = a22 + L::cs2 * tr;
    const R r1 = m.drho * L::w1, r5 = m.drho * L::w5;
    h[0] = fmadd(m.drho, L::w0, M22 - tr);
    const R u = a20 - M22, v = m.jx - M12;  // 2 (h1 - r1), 2 (h3 - r1) = u + v, u - v
    const R p = a02 - M22, q = m.jy - M21;
    h[1] = fmadd(R(0.5), u + v, r1);
    h[3] = fmadd(R(0.5), u - v, r1);
    h[2] = fmadd(R(0.5), p + q, r1);
    h[4] = fmadd(R(0.5), p - q, r1);
    const R A = M22 + a11, B = M22 - a11, C = M12 + M21, D = M12 - M21;
    h[5] = fmadd(R(0.25), A + C, r5);
    h[6] = fmadd(R(0.25), B - D, r5);
    h[7] = fmadd(R(0.25), A - C, r5);
    h[8] = fmadd(R(0.25), B + D, r5);
}

// Hermite non-equilibrium moments d_pq = A_pq - A^eq_pq of the shifted populations.
template <typename R> struct Neq {
    R d20, d02, d11, d21, d12, d22;
};

template <typename R>
__device__ __forceinline__ Neq<R> hermite_neq(const R (&h)[9], const Macro<R>& m, const Eq<R>& e) {
    using L = Lat<R>;
    const R s58 = h[5] + h[8], s67 = h[6] + h[7];
    const R diag = s58 + s67;                                  // m22
    const R m20 = (h[1] + h[3]) + diag;
    const R m02 = (h[2] + h[4]) + diag;
    const R m11 = (h[5] + h[7]) - (h[6] + h[8]);
    const R m21 = (h[5] + h[6]) - (h[7] + h[8]);
    const R m12 = s58 - s67;
    const R a20 = m20 - m.drho * L::cs2;
    const R a02 = m02 - m.drho * L::cs2;
    const R a22 = (diag - m.drho * L::cs4) - L::cs2 * (a20 + a02);
    Neq<R> d;
    d.d20 = a20 - e.e20;
    d.d02 = a02 - e.e02;
    d.d11 = m11 - e.e11;
    d.d21 = (m21 - L::cs2 * m.jy) - e.e21;
    d.d12 = (m12 - L::cs2 * m.jx) - e.e12;
    d.d22 = a22 - e.e22;
    return d;
}

// Collide one cell in place.  N is the equilibrium order (2, 3 or 4; CM, CHM and K use 4).
template <int MODEL, typename R>
__device__ __forceinline__ void collide(R (&h)[9], const Macro<R>& m, const Ref<R>& ref,
                                        const Coef<R>& c, int N) {
    using L = Lat<R>;
    if constexpr (MODEL == kStreamOnly) {
        return;
    } else {
        const Eq<R> e = hermite_eq(m, ref, N);
        if constexpr (MODEL == kBGK) {
            R heq[9];
            hermite_to_pop(m, e.e20, e.e02, e.e11, e.e21, e.e12, e.e22, heq);
#pragma unroll
            for (int i = 0; i < 9; ++i) h[i] = h[i] - c.om * (h[i] - heq[i]);
        } else {
            const Neq<R> d = hermite_neq(h, m, e);
            // second-order block, common to every moment space
            const R n20 = c.cpp * d.d20 + c.cpm * d.d02;
            const R n02 = c.cpm * d.d20 + c.cpp * d.d02;
            const R n11 = c.c11 * d.d11;
            R n21, n12, n22;
            if constexpr (MODEL == kHM || MODEL == kPR) {
                if constexpr (MODEL == kPR) {
                    n21 = R(0); n12 = R(0); n22 = R(0);
                } else {
                    n21 = c.c21 * d.d21;
                    n12 = c.c12 * d.d12;
                    n22 = c.c22 * d.d22;
                }
            } else if constexpr (MODEL == kRM) {
                // raw fourth-order moment: M22 - M22^eq = d22 + cs2 (d20 + d02)
                n21 = c.c21 * d.d21;
                n12 = c.c12 * d.d12;
                n22 = c.c22 * (d.d22 + L::cs2 * (d.d20 + d.d02)) - L::cs2 * (n20 + n02);
            } else if constexpr (MODEL == kRR) {
                // recursive non-equilibrium Hermite moments (eq. RRformulas_D2Q9)
                n21 = c.c21 * (m.uy * d.d20 + R(2) * m.ux * d.d11);
                n12 = c.c12 * (m.ux * d.d02 + R(2) * m.uy * d.d11);
                n22 = c.c22 * (m.uy * m.uy * d.d20 + m.ux * m.ux * d.d02 + R(4) * m.ux * m.uy * d.d11);
            } else {  // kCM, kCHM, kK: central Hermite moments t = shift(-u) of d
                const R ux = m.ux, uy = m.uy;
                const R t21 = d.d21 - uy * d.d20 - R(2) * ux * d.d11;
                const R t12 = d.d12 - ux * d.d02 - R(2) * uy * d.d11;
                const R t22 = d.d22 - R(2) * (uy * d.d21 + ux * d.d12) + uy * uy * d.d20 +
                              ux * ux * d.d02 + R(4) * ux * uy * d.d11;
                const R s21 = c.c21 * t21;
                const R s12 = c.c12 * t12;
                R s22;
                if constexpr (MODEL == kCHM) {
                    s22 = c.c22 * t22;
                } else if constexpr (MODEL == kCM) {
                    // central fourth-order moment: k22 - k22^eq = t22 + cs2 (t20 + t02)
                    s22 = c.c22 * (t22 + L::cs2 * (d.d20 + d.d02)) - L::cs2 * (n20 + n02);
                } else {
                    // fourth-order cumulant times rho: t22 - (t20 t02 + 2 t11^2) / rho
                    const R inv = m.inv_rho;
                    s22 = c.c22 * (t22 - (d.d20 * d.d02 + R(2) * d.d11 * d.d11) * inv) +
                          (n20 * n02 + R(2) * n11 * n11) * inv;
                }
                // back to Hermite moments (eq. CHM2HM_Q9, equilibrium parts cancel)
                n21 = s21 + uy * n20 + R(2) * ux * n11;
                n12 = s12 + ux * n02 + R(2) * uy * n11;
                n22 = s22 + R(2) * (uy * s21 + ux * s12) + uy * uy * n20 + ux * ux * n02 +
                      R(4) * ux * uy * n11;
            }
            hermite_to_pop(m, e.e20 + n20, e.e02 + n02, e.e11 + n11, e.e21 + n21, e.e12 + n12,
                           e.e22 + n22, h);
        }
    }
}

}  // namespace lbm
