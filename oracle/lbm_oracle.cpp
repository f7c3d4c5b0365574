// Plain FP64 CPU oracle of the D2Q9 stream-and-collide lattice Boltzmann method with the
// eight collision models compared by Coreixas, Wissocq, Chopard & Latt, "Impact of collision
// models on the physical properties and the stability of lattice Boltzmann methods" (2020).
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference the HIP path
// is checked against.  Only the test-suite, the smoke check and the benchmark's CPU-baseline
// leg may load it.  It shares no code, header, table or helper with the GPU library.
//
// Style: single-threaded, every moment is a literal sum over the nine populations, every map
// is written in the order and notation of the paper (Appendix B), no fusion or reordering.
// Built with -O2 -ffp-contract=off so the arithmetic is exactly what is written.
//
// Readings of the paper that are not printed there (each is pinned by a test):
//   * c_s^2 = 1/3 (lattice temperature T0 = c_s^2, Section 5.1 vortex initialisation).
//   * Equilibrium of order N in {2,3,4}: Hermite equilibrium moments A^eq_pq = rho ux^p uy^q
//     with A^eq_pq = 0 when p+q > N, mapped to raw moments by the HM->RM relations
//     (eq. HM2RM_Q9).  N = 4 is the extended (product-form) equilibrium of eq. extendedFeq,
//     whose raw moments are listed under eq. RMcoll (M22^eq = M20^eq M02^eq / rho).
//   * Five relaxation frequencies (omega_nu, omega_b, omega_21, omega_12, omega_22): the
//     second-order block is split into deviator (omega_nu) and trace (omega_b).  The paper's
//     (omega_nu, omega_3, omega_4) is the case omega_b = omega_nu, omega_21 = omega_12 =
//     omega_3, omega_22 = omega_4.
//   * CM: central-moment equilibrium {k00 = rho, k20 = k02 = rho cs^2, k22 = rho cs^4, others
//     0}; back-transform by the binomial shift of (xi - u) + u, which has the form of
//     eq. CHM2HM_Q9.
//   * K: cumulants of f/rho in the peculiar velocity; K22 = n22 - n20 n02 - 2 n11^2, all
//     other cumulants up to (2,2) equal the normalised central moments n_pq = k_pq / rho.
//   * RR (eq. HMColl_Q9): for third and fourth order the pre-collision Hermite moment is the
//     regularised one, A^eq + A^neq(recursive), so A*_pq = A^eq_pq + (1 - omega) A^neq_pq.
//   * PR is HM with omega_21 = omega_12 = omega_22 = 1 (standard regularisation).

#include <complex>
#include <cstddef>
#include <cstring>
#include <vector>

namespace {

using cplx = std::complex<double>;

constexpr int Q = 9;
// D2Q9 velocities xi_i = (xi_x, xi_y), index order (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),
// (-1,1),(-1,-1),(1,-1) (Section 2: xi_alpha in {0, +-1}).
constexpr int XI[Q][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                          {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
constexpr double CS2 = 1.0 / 3.0;

enum Model { BGK = 0, RM = 1, HM = 2, CM = 3, CHM = 4, K = 5, PR = 6, RR = 7, STREAM_ONLY = 99 };

// omega = (omega_nu, omega_b, omega_21, omega_12, omega_22)
enum { W_NU = 0, W_B = 1, W_21 = 2, W_12 = 3, W_22 = 4 };

template <class T>
struct Mom {  // X[p][q], p, q in {0, 1, 2}
    T v[3][3];
};

template <class T>
T ipow(T x, int p) {
    T r = T(1.0);
    for (int k = 0; k < p; ++k) r = r * x;
    return r;
}

// One-dimensional Hermite polynomial of order p at z with variance cs^2 (eq. CHpoly with
// u = 0 gives the Hermite polynomials, with u the central Hermite ones).
template <class T>
T herm1(int p, T z) {
    if (p == 0) return T(1.0);
    if (p == 1) return z;
    return z * z - T(CS2);
}

// Raw moments M_pq = sum_i xi_x^p xi_y^q f_i (definition under eq. RMcoll; the second
// exponent applies to xi_y).
template <class T>
Mom<T> raw_moments(const T f[Q]) {
    Mom<T> M;
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            T s = T(0.0);
            for (int i = 0; i < Q; ++i)
                s = s + ipow(T(double(XI[i][0])), p) * ipow(T(double(XI[i][1])), q) * f[i];
            M.v[p][q] = s;
        }
    return M;
}

// Hermite moments A_pq = sum_i H_pq(xi_i) f_i.
template <class T>
Mom<T> hermite_moments(const T f[Q]) {
    Mom<T> A;
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            T s = T(0.0);
            for (int i = 0; i < Q; ++i)
                s = s + herm1(p, T(double(XI[i][0]))) * herm1(q, T(double(XI[i][1]))) * f[i];
            A.v[p][q] = s;
        }
    return A;
}

// Central moments k_pq = sum_i (xi_x - ux)^p (xi_y - uy)^q f_i.
template <class T>
Mom<T> central_moments(const T f[Q], T ux, T uy) {
    Mom<T> k;
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            T s = T(0.0);
            for (int i = 0; i < Q; ++i)
                s = s + ipow(T(double(XI[i][0])) - ux, p) * ipow(T(double(XI[i][1])) - uy, q) * f[i];
            k.v[p][q] = s;
        }
    return k;
}

// Central Hermite moments A~_pq = sum_i H~_pq f_i (eq. CHpoly).
template <class T>
Mom<T> central_hermite_moments(const T f[Q], T ux, T uy) {
    Mom<T> A;
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            T s = T(0.0);
            for (int i = 0; i < Q; ++i)
                s = s + herm1(p, T(double(XI[i][0])) - ux) * herm1(q, T(double(XI[i][1])) - uy) * f[i];
            A.v[p][q] = s;
        }
    return A;
}

// Post-collision populations from raw moments (eq. Q9postCollVDF_RM), sigma = xi_x,
// lambda = xi_y.
template <class T>
void rm_to_f(const Mom<T>& M, T f[Q]) {
    const T M00 = M.v[0][0], M10 = M.v[1][0], M01 = M.v[0][1], M20 = M.v[2][0], M02 = M.v[0][2],
            M11 = M.v[1][1], M21 = M.v[2][1], M12 = M.v[1][2], M22 = M.v[2][2];
    for (int i = 0; i < Q; ++i) {
        const int sx = XI[i][0], sy = XI[i][1];
        const T sg = T(double(sx)), la = T(double(sy));
        if (sx == 0 && sy == 0)
            f[i] = M00 - (M20 + M02) + M22;
        else if (sy == 0)
            f[i] = T(0.5) * (sg * M10 + M20 - sg * M12 - M22);
        else if (sx == 0)
            f[i] = T(0.5) * (la * M01 + M02 - la * M21 - M22);
        else
            f[i] = T(0.25) * (sg * la * M11 + sg * M12 + la * M21 + M22);
    }
}

// Post-collision Hermite -> raw moments (eq. HM2RM_Q9).
template <class T>
Mom<T> hm_to_rm(const Mom<T>& A, T rho, T ux, T uy) {
    Mom<T> M;
    M.v[0][0] = A.v[0][0];
    M.v[1][0] = A.v[1][0];
    M.v[0][1] = A.v[0][1];
    M.v[1][1] = A.v[1][1];
    M.v[2][0] = A.v[2][0] + rho * T(CS2);
    M.v[0][2] = A.v[0][2] + rho * T(CS2);
    M.v[2][1] = A.v[2][1] + rho * T(CS2) * uy;
    M.v[1][2] = A.v[1][2] + rho * T(CS2) * ux;
    M.v[2][2] = A.v[2][2] + T(CS2) * (A.v[2][0] + A.v[0][2]) + rho * T(CS2 * CS2);
    return M;
}

// Shift of a centred set of moments T (T10 = T01 = 0) by the velocity u: this is the
// binomial expansion of ((xi - u) + u)^p, written in the form of eq. CHM2HM_Q9.  It maps
// central Hermite moments to Hermite moments, and central moments to raw moments.
template <class T>
Mom<T> shift_by_u(const Mom<T>& C, T rho, T ux, T uy) {
    Mom<T> R;
    R.v[0][0] = rho;
    R.v[1][0] = rho * ux;
    R.v[0][1] = rho * uy;
    R.v[2][0] = C.v[2][0] + rho * ux * ux;
    R.v[0][2] = C.v[0][2] + rho * uy * uy;
    R.v[1][1] = C.v[1][1] + rho * ux * uy;
    R.v[2][1] = C.v[2][1] + uy * C.v[2][0] + T(2.0) * ux * C.v[1][1] + rho * ux * ux * uy;
    R.v[1][2] = C.v[1][2] + ux * C.v[0][2] + T(2.0) * uy * C.v[1][1] + rho * ux * uy * uy;
    R.v[2][2] = C.v[2][2] + T(2.0) * uy * C.v[2][1] + T(2.0) * ux * C.v[1][2] + uy * uy * C.v[2][0] +
                ux * ux * C.v[0][2] + T(4.0) * ux * uy * C.v[1][1] + rho * ux * ux * uy * uy;
    return R;
}

// Hermite equilibrium moments of order N: A^eq_pq = rho ux^p uy^q for p+q <= N, else 0.
template <class T>
Mom<T> eq_hermite(T rho, T ux, T uy, int N) {
    Mom<T> A;
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q)
            A.v[p][q] = (p + q <= N) ? rho * ipow(ux, p) * ipow(uy, q) : T(0.0);
    return A;
}

// Raw equilibrium moments.  N = 4: the list under eq. RMcoll.  N < 4: truncated Hermite
// equilibrium mapped by eq. HM2RM_Q9.
template <class T>
Mom<T> eq_raw(T rho, T ux, T uy, int N) {
    if (N == 4) {
        Mom<T> M;
        M.v[0][0] = rho;
        M.v[1][0] = rho * ux;
        M.v[0][1] = rho * uy;
        M.v[2][0] = rho * (ux * ux + T(CS2));
        M.v[0][2] = rho * (uy * uy + T(CS2));
        M.v[1][1] = rho * ux * uy;
        M.v[2][1] = M.v[2][0] * uy;
        M.v[1][2] = ux * M.v[0][2];
        M.v[2][2] = M.v[2][0] * M.v[0][2] / rho;
        return M;
    }
    return hm_to_rm(eq_hermite(rho, ux, uy, N), rho, ux, uy);
}

// Discrete equilibrium f^eq (eq. extendedFeq, right-hand forms).
template <class T>
void feq(T rho, T ux, T uy, int N, T f[Q]) {
    rm_to_f(eq_raw(rho, ux, uy, N), f);
}

// Relaxation X* = X^eq + (1 - omega)(X - X^eq) of the six non-conserved moments (eq. RMcoll /
// eq. CHMcoll), the second-order diagonal pair split into trace (omega_b) and deviator
// (omega_nu).  Conserved moments X00, X10, X01 are copied.
template <class T>
Mom<T> relax(const Mom<T>& X, const Mom<T>& Xeq, const T w[5]) {
    Mom<T> Y = X;
    const T d20 = X.v[2][0] - Xeq.v[2][0];
    const T d02 = X.v[0][2] - Xeq.v[0][2];
    const T trace = d20 + d02;
    const T dev = d20 - d02;
    const T one = T(1.0);
    Y.v[2][0] = Xeq.v[2][0] + T(0.5) * ((one - w[W_B]) * trace + (one - w[W_NU]) * dev);
    Y.v[0][2] = Xeq.v[0][2] + T(0.5) * ((one - w[W_B]) * trace - (one - w[W_NU]) * dev);
    Y.v[1][1] = Xeq.v[1][1] + (one - w[W_NU]) * (X.v[1][1] - Xeq.v[1][1]);
    Y.v[2][1] = Xeq.v[2][1] + (one - w[W_21]) * (X.v[2][1] - Xeq.v[2][1]);
    Y.v[1][2] = Xeq.v[1][2] + (one - w[W_12]) * (X.v[1][2] - Xeq.v[1][2]);
    Y.v[2][2] = Xeq.v[2][2] + (one - w[W_22]) * (X.v[2][2] - Xeq.v[2][2]);
    return Y;
}

// Density and velocity: rho = M00, rho u = (M10, M01) (eq. RMcoll, conserved moments).
template <class T>
void macroscopic(const T f[Q], T& rho, T& ux, T& uy) {
    const Mom<T> M = raw_moments(f);
    rho = M.v[0][0];
    ux = M.v[1][0] / rho;
    uy = M.v[0][1] / rho;
}

// Post-collision populations of one cell.
template <class T>
int collide(int model, int N, const T w_in[5], const T f[Q], T fs[Q]) {
    T w[5];
    for (int k = 0; k < 5; ++k) w[k] = w_in[k];
    if (model == STREAM_ONLY) {
        for (int i = 0; i < Q; ++i) fs[i] = f[i];
        return 0;
    }
    T rho, ux, uy;
    macroscopic(f, rho, ux, uy);
    switch (model) {
        case BGK: {  // f* = f - omega_nu (f - f^eq)
            T fe[Q];
            feq(rho, ux, uy, N, fe);
            for (int i = 0; i < Q; ++i) fs[i] = f[i] - w[W_NU] * (f[i] - fe[i]);
            return 0;
        }
        case RM: {  // relax raw moments, eq. RMcoll, then eq. Q9postCollVDF_RM
            const Mom<T> M = raw_moments(f);
            const Mom<T> Ms = relax(M, eq_raw(rho, ux, uy, N), w);
            rm_to_f(Ms, fs);
            return 0;
        }
        case PR:  // standard regularisation: HM with equilibrated high-order moments
            w[W_21] = T(1.0);
            w[W_12] = T(1.0);
            w[W_22] = T(1.0);
            /* fall through */
        case HM: {  // relax Hermite moments, then HM -> RM -> f
            const Mom<T> A = hermite_moments(f);
            const Mom<T> As = relax(A, eq_hermite(rho, ux, uy, N), w);
            rm_to_f(hm_to_rm(As, rho, ux, uy), fs);
            return 0;
        }
        case CM: {  // relax central moments, shift to raw moments, then f
            if (N != 4) return -2;
            const Mom<T> k = central_moments(f, ux, uy);
            Mom<T> keq;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) keq.v[p][q] = T(0.0);
            keq.v[0][0] = rho;
            keq.v[2][0] = rho * T(CS2);
            keq.v[0][2] = rho * T(CS2);
            keq.v[2][2] = rho * T(CS2 * CS2);
            const Mom<T> ks = relax(k, keq, w);
            rm_to_f(shift_by_u(ks, rho, ux, uy), fs);
            return 0;
        }
        case CHM: {  // eq. CHMcoll, eq. CHM2HM_Q9, eq. HM2RM_Q9, eq. Q9postCollVDF_RM
            if (N != 4) return -2;
            const Mom<T> At = central_hermite_moments(f, ux, uy);
            Mom<T> Ateq;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) Ateq.v[p][q] = T(0.0);
            Ateq.v[0][0] = rho;
            const Mom<T> Ats = relax(At, Ateq, w);
            const Mom<T> As = shift_by_u(Ats, rho, ux, uy);
            rm_to_f(hm_to_rm(As, rho, ux, uy), fs);
            return 0;
        }
        case K: {  // cumulants of f / rho in the peculiar velocity
            if (N != 4) return -2;
            const Mom<T> k = central_moments(f, ux, uy);
            Mom<T> n;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) n.v[p][q] = k.v[p][q] / rho;
            Mom<T> C = n;  // cumulants
            C.v[2][2] = n.v[2][2] - n.v[2][0] * n.v[0][2] - T(2.0) * n.v[1][1] * n.v[1][1];
            Mom<T> Ceq;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) Ceq.v[p][q] = T(0.0);
            Ceq.v[0][0] = T(1.0);
            Ceq.v[2][0] = T(CS2);
            Ceq.v[0][2] = T(CS2);
            const Mom<T> Cs = relax(C, Ceq, w);
            Mom<T> ns = Cs;  // back to normalised central moments
            ns.v[2][2] = Cs.v[2][2] + Cs.v[2][0] * Cs.v[0][2] + T(2.0) * Cs.v[1][1] * Cs.v[1][1];
            Mom<T> ks;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) ks.v[p][q] = rho * ns.v[p][q];
            rm_to_f(shift_by_u(ks, rho, ux, uy), fs);
            return 0;
        }
        case RR: {  // eq. HMColl_Q9 with the recursive non-equilibrium moments of eq. RRformulas_D2Q9
            const Mom<T> A = hermite_moments(f);
            const Mom<T> Aeq = eq_hermite(rho, ux, uy, N);
            Mom<T> Aneq;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) Aneq.v[p][q] = T(0.0);
            Aneq.v[2][0] = A.v[2][0] - Aeq.v[2][0];
            Aneq.v[0][2] = A.v[0][2] - Aeq.v[0][2];
            Aneq.v[1][1] = A.v[1][1] - Aeq.v[1][1];
            Aneq.v[2][1] = uy * Aneq.v[2][0] + T(2.0) * ux * Aneq.v[1][1];
            Aneq.v[1][2] = ux * Aneq.v[0][2] + T(2.0) * uy * Aneq.v[1][1];
            Aneq.v[2][2] = uy * uy * Aneq.v[2][0] + ux * ux * Aneq.v[0][2] + T(4.0) * ux * uy * Aneq.v[1][1];
            Mom<T> Areg;  // regularised Hermite moments A^eq + A^neq
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) Areg.v[p][q] = Aeq.v[p][q] + Aneq.v[p][q];
            Areg.v[0][0] = rho;
            Areg.v[1][0] = rho * ux;
            Areg.v[0][1] = rho * uy;
            const Mom<T> As = relax(Areg, Aeq, w);
            rm_to_f(hm_to_rm(As, rho, ux, uy), fs);
            return 0;
        }
        default:
            return -1;
    }
}

inline size_t idx(int q, int x, int y, int nx, int ny) {
    return (size_t(q) * size_t(ny) + size_t(y)) * size_t(nx) + size_t(x);
}

inline int wrap(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

}  // namespace

extern "C" {

// Populations are stored f[q][y][x] (x fastest), q in the index order of XI.
int oracle_q(void) { return Q; }

void oracle_velocities(int* cx, int* cy) {
    for (int i = 0; i < Q; ++i) {
        cx[i] = XI[i][0];
        cy[i] = XI[i][1];
    }
}

// One cell's post-collision populations.  Returns 0, -1 (unknown model) or -2 (model needs
// N = 4).
int oracle_collide_cell(int model, int N, const double* omega, const double* f, double* fs) {
    return collide<double>(model, N, omega, f, fs);
}

void oracle_feq_cell(int N, double rho, double ux, double uy, double* f) {
    feq<double>(rho, ux, uy, N, f);
}

// Moments of one cell: kind 0 raw, 1 Hermite, 2 central, 3 central Hermite; out[3*p+q].
void oracle_moments_cell(int kind, const double* f, double* out) {
    double rho, ux, uy;
    macroscopic(f, rho, ux, uy);
    Mom<double> m;
    if (kind == 0)
        m = raw_moments(f);
    else if (kind == 1)
        m = hermite_moments(f);
    else if (kind == 2)
        m = central_moments(f, ux, uy);
    else
        m = central_hermite_moments(f, ux, uy);
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) out[3 * p + q] = m.v[p][q];
}

// f = f^eq_N(rho, u) on every node.  rho, ux, uy are [y][x].
void oracle_init_eq(int nx, int ny, int N, const double* rho, const double* ux, const double* uy,
                    double* f) {
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t c = size_t(y) * nx + x;
            double fe[Q];
            feq<double>(rho[c], ux[c], uy[c], N, fe);
            for (int i = 0; i < Q; ++i) f[idx(i, x, y, nx, ny)] = fe[i];
        }
}

// nsteps of collide-then-stream on a periodic nx x ny grid (eq. StreamCollide):
// f_i(x + xi_i, t + 1) = f*_i(x, t).  f holds the pre-collision state and is updated in place
// (a second buffer is allocated internally).  Returns the collide status.
int oracle_step(int nx, int ny, int model, int N, const double* omega, double* f, int nsteps) {
    std::vector<double> g(size_t(Q) * nx * ny);
    for (int s = 0; s < nsteps; ++s) {
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double fc[Q], fs[Q];
                for (int i = 0; i < Q; ++i) fc[i] = f[idx(i, x, y, nx, ny)];
                const int rc = collide<double>(model, N, omega, fc, fs);
                if (rc != 0) return rc;
                for (int i = 0; i < Q; ++i)
                    g[idx(i, wrap(x + XI[i][0], nx), wrap(y + XI[i][1], ny), nx, ny)] = fs[i];
            }
        std::memcpy(f, g.data(), g.size() * sizeof(double));
    }
    return 0;
}

// Macroscopic fields and totals of a state: rho, ux, uy ([y][x], may be null) and
// totals = {sum rho, sum rho ux, sum rho uy, sum 0.5 rho |u|^2, mean |u|^2}.
void oracle_moments(int nx, int ny, const double* f, double* rho, double* ux, double* uy,
                    double* totals) {
    double t[5] = {0, 0, 0, 0, 0};
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double fc[Q];
            for (int i = 0; i < Q; ++i) fc[i] = f[idx(i, x, y, nx, ny)];
            double r, u, v;
            macroscopic(fc, r, u, v);
            const size_t c = size_t(y) * nx + x;
            if (rho) rho[c] = r;
            if (ux) ux[c] = u;
            if (uy) uy[c] = v;
            t[0] += r;
            t[1] += r * u;
            t[2] += r * v;
            t[3] += 0.5 * r * (u * u + v * v);
            t[4] += u * u + v * v;
        }
    t[4] /= double(nx) * double(ny);
    if (totals)
        for (int k = 0; k < 5; ++k) totals[k] = t[k];
}

// Jacobians of one cell's collision by the complex-step derivative (Squire & Trapp 1998):
// dC_i/dz = Im C_i(z + i h) / h, exact to rounding because the collision is a rational
// function of f and omega.  J[9*i + j] = dC_i/df_j, Jw[5*i + k] = dC_i/domega_k.
int oracle_collide_jacobian(int model, int N, const double* omega, const double* f, double* J,
                            double* Jw) {
    const double h = 1e-30;
    cplx fc[Q], wc[5], out[Q];
    for (int j = 0; j < Q + 5; ++j) {
        for (int i = 0; i < Q; ++i) fc[i] = cplx(f[i], 0.0);
        for (int k = 0; k < 5; ++k) wc[k] = cplx(omega[k], 0.0);
        if (j < Q)
            fc[j] = cplx(f[j], h);
        else
            wc[j - Q] = cplx(omega[j - Q], h);
        const int rc = collide<cplx>(model, N, wc, fc, out);
        if (rc != 0) return rc;
        for (int i = 0; i < Q; ++i) {
            if (j < Q) {
                if (J) J[Q * i + j] = out[i].imag() / h;
            } else {
                if (Jw) Jw[5 * i + (j - Q)] = out[i].imag() / h;
            }
        }
    }
    return 0;
}

// Derivatives of f^eq_N with respect to (ux, uy) at fixed rho, by complex step:
// d[2*i + a] = df^eq_i / du_a.
void oracle_feq_jacobian(int N, double rho, double ux, double uy, double* d) {
    const double h = 1e-30;
    cplx out[Q];
    feq<cplx>(cplx(rho, 0.0), cplx(ux, h), cplx(uy, 0.0), N, out);
    for (int i = 0; i < Q; ++i) d[2 * i + 0] = out[i].imag() / h;
    feq<cplx>(cplx(rho, 0.0), cplx(ux, 0.0), cplx(uy, h), N, out);
    for (int i = 0; i < Q; ++i) d[2 * i + 1] = out[i].imag() / h;
}

// One reverse step of the discrete adjoint of f_{n+1} = S C(f_n):
//   mu_i(x) = lam_next_i(x + xi_i)          (transpose of the streaming permutation)
//   lam_i(x) = sum_j dC_j/df_i (f_n(x)) mu_j(x)
//   domega_k += sum_x sum_j dC_j/domega_k mu_j(x)
// f_n is the pre-collision state of step n; all arrays are [q][y][x].
int oracle_adjoint_step(int nx, int ny, int model, int N, const double* omega, const double* f_n,
                        const double* lam_next, double* lam, double* domega) {
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double fc[Q], mu[Q], J[Q * Q], Jw[Q * 5];
            for (int i = 0; i < Q; ++i) {
                fc[i] = f_n[idx(i, x, y, nx, ny)];
                mu[i] = lam_next[idx(i, wrap(x + XI[i][0], nx), wrap(y + XI[i][1], ny), nx, ny)];
            }
            const int rc = oracle_collide_jacobian(model, N, omega, fc, J, Jw);
            if (rc != 0) return rc;
            for (int i = 0; i < Q; ++i) {
                double s = 0.0;
                for (int j = 0; j < Q; ++j) s += J[Q * j + i] * mu[j];
                lam[idx(i, x, y, nx, ny)] = s;
            }
            for (int k = 0; k < 5; ++k) {
                double s = 0.0;
                for (int j = 0; j < Q; ++j) s += Jw[5 * j + k] * mu[j];
                domega[k] += s;
            }
        }
    return 0;
}

// Pull-back of the initial-state adjoint to the initial velocity field:
// du_a(x) = sum_i df^eq_i/du_a (rho(x), u(x)) lam0_i(x).
void oracle_feq_vjp(int nx, int ny, int N, const double* rho, const double* ux, const double* uy,
                    const double* lam0, double* dux, double* duy) {
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t c = size_t(y) * nx + x;
            double d[2 * Q];
            oracle_feq_jacobian(N, rho[c], ux[c], uy[c], d);
            double sx = 0.0, sy = 0.0;
            for (int i = 0; i < Q; ++i) {
                sx += d[2 * i + 0] * lam0[idx(i, x, y, nx, ny)];
                sy += d[2 * i + 1] * lam0[idx(i, x, y, nx, ny)];
            }
            dux[c] = sx;
            duy[c] = sy;
        }
}

}  // extern "C"
