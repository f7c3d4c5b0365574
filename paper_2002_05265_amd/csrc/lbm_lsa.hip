// Linear stability analysis (lbm_lsa.h): the collision Jacobian J_C about a uniform flow, and the
// eigenvalues of M(k) = diag(exp(-i xi_i . k)) J_C for many wave numbers at once.
//
// J_C comes from the reverse mode of the library's own collision (lbm_adjoint_cell.hpp): with the
// adjoint seed mu = e_i, collide_adjoint returns J_C^T e_i, i.e. row i of J_C.  The eigenvalues of
// each 9 x 9 complex M(k) are found by one thread: Givens reduction to upper Hessenberg form,
// then implicit single-shift QR sweeps (Wilkinson shift from the trailing 2 x 2 block, Givens
// rotations chasing the bulge) with deflation of negligible subdiagonal entries, the matrix held
// in registers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "lbm.h"
#include "lbm_lsa.h"
#include "lbm_cell.hpp"
#include "lbm_internal.hpp"
#include "lbm_adjoint_cell.hpp"

using namespace lbm;

namespace {

constexpr int kQ = 9;

struct cplx {
    double re, im;
};
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.re, -a.im}; }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ double cabs(cplx a) { return hypot(a.re, a.im); }
__device__ __forceinline__ cplx csqrt(cplx a) {
    // principal square root
    const double r = cabs(a);
    if (r == 0.0) return {0.0, 0.0};
    const double t = sqrt(0.5 * (r + fabs(a.re)));
    if (a.re >= 0.0) return {t, a.im / (2.0 * t)};
    return {fabs(a.im) / (2.0 * t), a.im >= 0.0 ? t : -t};
}

// Reverse-mode collision of one cell, dispatched on the model at run time.
__device__ void collide_adjoint_model(int model, const double (&h)[9], const Macro<double>& m,
                                      const Ref<double>& r, const Coef<double>& c, int N, const double (&mu)[9],
                                      double (&hb)[9], double (&cb)[7]) {
    switch (model) {
        case kBGK: collide_adjoint<kBGK>(h, m, r, c, N, mu, hb, cb); break;
        case kRM: collide_adjoint<kRM>(h, m, r, c, N, mu, hb, cb); break;
        case kHM: collide_adjoint<kHM>(h, m, r, c, N, mu, hb, cb); break;
        case kCM: collide_adjoint<kCM>(h, m, r, c, N, mu, hb, cb); break;
        case kCHM: collide_adjoint<kCHM>(h, m, r, c, N, mu, hb, cb); break;
        case kK: collide_adjoint<kK>(h, m, r, c, N, mu, hb, cb); break;
        case kPR: collide_adjoint<kPR>(h, m, r, c, N, mu, hb, cb); break;
        default: collide_adjoint<kRR>(h, m, r, c, N, mu, hb, cb); break;
    }
}

// Row i = threadIdx.x of J_C for point blockIdx.x.
__global__ void k_lsa_jacobian(const lbm_lsa_point* __restrict__ pts, double* __restrict__ J) {
    const int p = blockIdx.x, i = threadIdx.x;
    if (i >= kQ) return;
    const lbm_lsa_point& q = pts[p];
    const Ref<double> ref{0.0, 0.0, 0.0};  // FP64: populations stored unshifted
    double h[9];
    eq_deviation(1.0, q.ux, q.uy, ref, q.eq_order, h);
    double rho_d;
    const Macro<double> m = macro_of<double>(h, ref, rho_d);
    const Coef<double> c = make_coef<double>(q.omega);
    double mu[9], hb[9], cb[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 9; ++j) mu[j] = j == i ? 1.0 : 0.0;
    collide_adjoint_model(q.model, h, m, ref, c, q.eq_order, mu, hb, cb);
#pragma unroll
    for (int j = 0; j < 9; ++j) J[(size_t)p * 81 + i * 9 + j] = hb[j];
}

// Every loop of the eigenvalue solver has bounds known at compile time (the active block's end
// HI is a template parameter, its start l a run-time value that predicates the rotations), so
// the matrix stays in registers: with run-time bounds it was indexed dynamically and lived in
// scratch memory, which bounded the kernel by scratch traffic.

// Rotation G = [c s; -conj(s) c] (c real) with G (x, y)^T = (r, 0)^T.
__device__ __forceinline__ void givens(cplx x, cplx y, double& c, cplx& sn) {
    const double r = sqrt(cabs2(x) + cabs2(y));
    if (r == 0.0) {
        c = 1.0;
        sn = {0.0, 0.0};
        return;
    }
    const double ax = cabs(x);
    if (ax == 0.0) {
        c = 0.0;
        sn = cscale(cconj(y), 1.0 / cabs(y));
    } else {
        c = ax / r;
        sn = cscale(cmul(cscale(x, 1.0 / ax), cconj(y)), 1.0 / r);
    }
}

// H <- G H G^H with G acting on rows / columns p, p + 1; the row rotation is applied to columns
// J0.. only (the entries left of J0 are zero in both rows), the column rotation to rows ..I1.
template <int P, int J0, int I1>
__device__ __forceinline__ void rotate(cplx (&H)[kQ][kQ], double c, cplx sn) {
#pragma unroll
    for (int jj = J0; jj < kQ; ++jj) {
        const cplx a = H[P][jj], b = H[P + 1][jj];
        H[P][jj] = cadd(cscale(a, c), cmul(sn, b));
        H[P + 1][jj] = csub(cscale(b, c), cmul(cconj(sn), a));
    }
#pragma unroll
    for (int i = 0; i <= I1; ++i) {
        const cplx a = H[i][P], b = H[i][P + 1];
        H[i][P] = cadd(cscale(a, c), cmul(b, cconj(sn)));
        H[i][P + 1] = csub(cscale(b, c), cmul(a, sn));
    }
}

// Reduction to upper Hessenberg form by Givens rotations: column K is cleared below its
// subdiagonal from the bottom up, each rotation of rows I - 1, I applied as a similarity (a
// rotation touches two rows and two columns, so few values are live beyond the matrix).
template <int K, int I>
__device__ __forceinline__ void hessenberg_col(cplx (&H)[kQ][kQ]) {
    if constexpr (I >= K + 2) {
        double c;
        cplx sn;
        givens(H[I - 1][K], H[I][K], c, sn);
        rotate<I - 1, K, kQ - 1>(H, c, sn);
        H[I][K] = {0.0, 0.0};
        // keep the scheduler from interleaving rotations, which would hold two copies of the
        // touched rows and columns and overflow the registers
        __builtin_amdgcn_sched_barrier(0);
        hessenberg_col<K, I - 1>(H);
    }
}

// Implicit single-shift QR iterations on the unreduced block l..HI (l found each iteration)
// until H[HI][HI-1] is negligible; then lam[HI] = H[HI][HI].  False if 90 iterations do not
// suffice.
template <int HI>
__device__ __forceinline__ bool converge_last(cplx (&H)[kQ][kQ], cplx (&lam)[kQ], double hnorm) {
    constexpr double eps = 2.220446049250313e-16;
    for (int its = 0;; ++its) {
        // start l of the unreduced block ending at HI: the last negligible subdiagonal entry
        int l = 0;
#pragma unroll
        for (int k = HI; k >= 1; --k) {
            double sdiag = cabs(H[k - 1][k - 1]) + cabs(H[k][k]);
            if (sdiag == 0.0) sdiag = hnorm;
            if (l == 0 && cabs(H[k][k - 1]) <= 2.0 * eps * sdiag) l = k;
        }
#pragma unroll
        for (int k = 1; k <= HI; ++k)
            if (k == l) H[k][k - 1] = {0.0, 0.0};
        if (l == HI) {
            lam[HI] = H[HI][HI];
            return true;
        }
        if (its >= 90) return false;
        // Wilkinson shift: eigenvalue of the trailing 2 x 2 block closer to H[HI][HI]
        cplx mu;
        const int it1 = its + 1;
        if (it1 % 30 == 10 || it1 % 30 == 20) {  // exceptional shift
            mu = cadd(H[HI][HI], cplx{0.75 * cabs(H[HI][HI - 1]), 0.0});
        } else {
            const cplx a = H[HI - 1][HI - 1], b = H[HI - 1][HI], c = H[HI][HI - 1], d = H[HI][HI];
            const cplx half = cscale(csub(a, d), 0.5);
            const cplx disc = csqrt(cadd(cmul(half, half), cmul(b, c)));
            const cplx m1 = cadd(d, csub(half, disc)), m2 = cadd(d, cadd(half, disc));
            mu = cabs2(csub(m1, d)) <= cabs2(csub(m2, d)) ? m1 : m2;
        }
        // first rotation from (H[l][l] - mu, H[l+1][l])
        cplx x = {0.0, 0.0}, y = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < HI; ++k)
            if (k == l) {
                x = csub(H[k][k], mu);
                y = H[k + 1][k];
            }
        // bulge chase over rows / columns l..HI.  The column rotations also touch the rows above
        // l (the coupling to the block above): a similarity of the whole matrix, which keeps it
        // block upper triangular, so no eigenvalue changes.
#pragma unroll
        for (int k = 0; k < HI; ++k) {
            if (k >= l) {
                double c;
                cplx sn;
                givens(x, y, c, sn);
                // rows k, k+1: [c s; -conj(s) c]  (entries left of column k - 1 are zero)
#pragma unroll
                for (int jj = (k > 0 ? k - 1 : 0); jj <= HI; ++jj) {
                    const cplx a = H[k][jj], b = H[k + 1][jj];
                    H[k][jj] = cadd(cscale(a, c), cmul(sn, b));
                    H[k + 1][jj] = csub(cscale(b, c), cmul(cconj(sn), a));
                }
                // columns k, k+1 (similarity with the conjugate transpose)
#pragma unroll
                for (int i = 0; i <= (k + 2 < HI ? k + 2 : HI); ++i) {
                    const cplx a = H[i][k], b = H[i][k + 1];
                    H[i][k] = cadd(cscale(a, c), cmul(b, cconj(sn)));
                    H[i][k + 1] = csub(cscale(b, c), cmul(a, sn));
                }
                if (k < HI - 1) {
                    x = H[k + 1][k];
                    y = H[k + 2][k];
                }
            }
        }
    }
}

// Eigenvalues of the 9 x 9 complex matrix H (overwritten).  Returns false if an eigenvalue did
// not converge within the iteration limit.
__device__ __forceinline__ bool eig9(cplx (&H)[kQ][kQ], cplx (&lam)[kQ]) {
    hessenberg_col<0, kQ - 1>(H);
    hessenberg_col<1, kQ - 1>(H);
    hessenberg_col<2, kQ - 1>(H);
    hessenberg_col<3, kQ - 1>(H);
    hessenberg_col<4, kQ - 1>(H);
    hessenberg_col<5, kQ - 1>(H);
    hessenberg_col<6, kQ - 1>(H);
    double hnorm = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; ++i)
#pragma unroll
        for (int jj = (i > 0 ? i - 1 : 0); jj < kQ; ++jj) hnorm = fmax(hnorm, cabs(H[i][jj]));
    bool ok = converge_last<8>(H, lam, hnorm);
    ok = ok && converge_last<7>(H, lam, hnorm);
    ok = ok && converge_last<6>(H, lam, hnorm);
    ok = ok && converge_last<5>(H, lam, hnorm);
    ok = ok && converge_last<4>(H, lam, hnorm);
    ok = ok && converge_last<3>(H, lam, hnorm);
    ok = ok && converge_last<2>(H, lam, hnorm);
    ok = ok && converge_last<1>(H, lam, hnorm);
    lam[0] = H[0][0];
    return ok;
}

// M(k) = diag(exp(-i xi . k)) J for wave number (kx, ky).  The nine phases are products of
// exp(-i kx) and exp(-i ky) (or their conjugates): two sincos calls, made before any entry of
// the matrix is live.
__device__ __forceinline__ void build_m(const double* __restrict__ J, double kx, double ky, cplx (&H)[kQ][kQ]) {
    double sx, cxk, sy, cyk;
    sincos(kx, &sx, &cxk);
    sincos(ky, &sy, &cyk);
    const cplx ex = {cxk, -sx}, ey = {cyk, -sy};  // exp(-i kx), exp(-i ky)
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const cplx px = cx(i) == 0 ? cplx{1.0, 0.0} : (cx(i) > 0 ? ex : cconj(ex));
        const cplx py = cy(i) == 0 ? cplx{1.0, 0.0} : (cy(i) > 0 ? ey : cconj(ey));
        const cplx ph = cmul(px, py);
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
            const double v = J[i * 9 + j];
            H[i][j] = {ph.re * v, ph.im * v};
        }
    }
}

__global__ __launch_bounds__(64) void k_lsa_radius(const double* __restrict__ J, int npts, const double* __restrict__ kx,
                                                   const double* __restrict__ ky, int nk, double* __restrict__ radius) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)npts * nk) return;
    const int p = (int)(idx / nk), q = (int)(idx - (long long)p * nk);
    cplx H[kQ][kQ], lam[kQ];
    build_m(J + (size_t)p * 81, kx[q], ky[q], H);
    double r = NAN;
    if (eig9(H, lam)) {
        r = 0.0;
#pragma unroll
        for (int m = 0; m < kQ; ++m) r = fmax(r, cabs(lam[m]));
    }
    radius[idx] = r;
}

__global__ __launch_bounds__(64) void k_lsa_eigenvalues(const double* __restrict__ J, const double* __restrict__ kx,
                                                        const double* __restrict__ ky, int nk, double* __restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nk) return;
    cplx H[kQ][kQ], lam[kQ];
    build_m(J, kx[q], ky[q], H);
    const bool ok = eig9(H, lam);
#pragma unroll
    for (int m = 0; m < kQ; ++m) {
        out[((size_t)q * kQ + m) * 2] = ok ? lam[m].re : NAN;
        out[((size_t)q * kQ + m) * 2 + 1] = ok ? lam[m].im : NAN;
    }
}

// M^C(k) = diag(xi . k) + i J^C, J^C = -(I - F) / tau, for the discrete-velocity Boltzmann
// equation with BGK collisions; F = d f^eq / d f at the base flow (the Jacobian of the BGK
// collision at omega = 1, whose post-collision state is f^eq).
__device__ __forceinline__ void build_dvbe(const double* __restrict__ F, double inv_tau, double kx, double ky,
                                           cplx (&H)[kQ][kQ]) {
#pragma unroll
    for (int i = 0; i < kQ; ++i)
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
            const double re = i == j ? (double)cx(i) * kx + (double)cy(i) * ky : 0.0;
            H[i][j] = {re, -inv_tau * ((i == j ? 1.0 : 0.0) - F[i * 9 + j])};
        }
}

// Largest growth rate max_m Im(omega_m) of a plane wave exp(i (k . x - omega t)) of the DVBE,
// omega the eigenvalues of M^C(k), for every (point, wave number) pair.
__global__ __launch_bounds__(64) void k_lsa_dvbe(const double* __restrict__ F, int npts, double inv_tau,
                                                 const double* __restrict__ kx, const double* __restrict__ ky,
                                                 int nk, double* __restrict__ growth) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)npts * nk) return;
    const int p = (int)(idx / nk), q = (int)(idx - (long long)p * nk);
    cplx H[kQ][kQ], lam[kQ];
    build_dvbe(F + (size_t)p * 81, inv_tau, kx[q], ky[q], H);
    double g = NAN;
    if (eig9(H, lam)) {
        g = -INFINITY;
#pragma unroll
        for (int m = 0; m < kQ; ++m) g = fmax(g, lam[m].im);
    }
    growth[idx] = g;
}

int check_points(const lbm_lsa_point* pts, int npts) {
    if (!pts || npts < 1) return set_error(LBM_EINVAL, "need npts >= 1 points");
    for (int p = 0; p < npts; ++p) {
        const lbm_lsa_point& q = pts[p];
        if (q.model < LBM_BGK || q.model > LBM_RR) return set_error(LBM_EINVAL, "point %d: model %d", p, q.model);
        if (q.eq_order < 2 || q.eq_order > 4) return set_error(LBM_EINVAL, "point %d: eq_order %d", p, q.eq_order);
        int rc = validate_model(q.model, q.eq_order);
        if (rc == LBM_OK) rc = validate_omega(q.omega);
        if (rc != LBM_OK) return rc;
        if (!(q.ux * q.ux + q.uy * q.uy < 1.0)) return set_error(LBM_EINVAL, "point %d: |U| must be < 1", p);
    }
    return LBM_OK;
}

// Copy the points to the device and compute their Jacobians into d_J (npts * 81 doubles).
int jacobians(const lbm_lsa_point* pts, int npts, double* d_J, hipStream_t s) {
    lbm_lsa_point* d_pts = nullptr;
    int rc = check_hip(hipMalloc(&d_pts, sizeof(lbm_lsa_point) * (size_t)npts), "hipMalloc(points)");
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpyAsync(d_pts, pts, sizeof(lbm_lsa_point) * (size_t)npts, hipMemcpyHostToDevice, s),
                       "copy points");
    if (rc == LBM_OK) {
        hipLaunchKernelGGL(k_lsa_jacobian, dim3(npts), dim3(64), 0, s, d_pts, d_J);
        rc = check_hip(hipGetLastError(), "jacobian launch");
    }
    if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(s), "synchronise");
    if (d_pts) (void)hipFree(d_pts);
    return rc;
}

}  // namespace

extern "C" {

int lbm_lsa_jacobian(const lbm_lsa_point* pts, int npts, double* J, void* hip_stream) {
    int rc = check_points(pts, npts);
    if (rc != LBM_OK) return rc;
    if (!J) return set_error(LBM_EINVAL, "J is NULL");
    return jacobians(pts, npts, J, static_cast<hipStream_t>(hip_stream));
}

int lbm_lsa_eigenvalues(const lbm_lsa_point* pt, const double* kx, const double* ky, int nk, double* lam,
                        void* hip_stream) {
    int rc = check_points(pt, 1);
    if (rc != LBM_OK) return rc;
    if (!kx || !ky || !lam) return set_error(LBM_EINVAL, "NULL pointer");
    if (nk < 1) return set_error(LBM_EINVAL, "nk %d < 1", nk);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    double* d_J = nullptr;
    rc = check_hip(hipMalloc(&d_J, sizeof(double) * 81), "hipMalloc(J)");
    if (rc == LBM_OK) rc = jacobians(pt, 1, d_J, s);
    if (rc == LBM_OK) {
        hipLaunchKernelGGL(k_lsa_eigenvalues, dim3((nk + 63) / 64), dim3(64), 0, s, d_J, kx, ky, nk, lam);
        rc = check_hip(hipGetLastError(), "eigenvalue launch");
    }
    if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(s), "synchronise");
    if (d_J) (void)hipFree(d_J);
    return rc;
}

int lbm_lsa_radius(const lbm_lsa_point* pts, int npts, const double* kx, const double* ky, int nk, double* radius,
                   void* hip_stream) {
    int rc = check_points(pts, npts);
    if (rc != LBM_OK) return rc;
    if (!kx || !ky || !radius) return set_error(LBM_EINVAL, "NULL pointer");
    if (nk < 1) return set_error(LBM_EINVAL, "nk %d < 1", nk);
    const long long total = (long long)npts * nk;
    if (total >= (1LL << 31)) return set_error(LBM_EINVAL, "npts * nk = %lld too large (one launch)", total);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    double* d_J = nullptr;
    rc = check_hip(hipMalloc(&d_J, sizeof(double) * 81 * (size_t)npts), "hipMalloc(J)");
    if (rc == LBM_OK) rc = jacobians(pts, npts, d_J, s);
    if (rc == LBM_OK) {
        hipLaunchKernelGGL(k_lsa_radius, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, s, d_J, npts, kx, ky, nk,
                           radius);
        rc = check_hip(hipGetLastError(), "radius launch");
    }
    if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(s), "synchronise");
    if (d_J) (void)hipFree(d_J);
    return rc;
}

int lbm_lsa_dvbe_growth(const lbm_lsa_point* pts, int npts, double tau, const double* kx, const double* ky,
                        int nk, double* growth, void* hip_stream) {
    if (!pts || npts < 1) return set_error(LBM_EINVAL, "need npts >= 1 points");
    if (!(tau > 0.0)) return set_error(LBM_EINVAL, "tau %g must be > 0", tau);
    if (!kx || !ky || !growth) return set_error(LBM_EINVAL, "NULL pointer");
    if (nk < 1) return set_error(LBM_EINVAL, "nk %d < 1", nk);
    const long long total = (long long)npts * nk;
    if (total >= (1LL << 31)) return set_error(LBM_EINVAL, "npts * nk = %lld too large (one launch)", total);
    // F = d f^eq / d f: the BGK collision's Jacobian at omega = 1, at each point's flow and order
    std::vector<lbm_lsa_point> bgk(pts, pts + npts);
    for (auto& q : bgk) {
        q.model = LBM_BGK;
        for (int k = 0; k < LBM_NOMEGA; ++k) q.omega[k] = 1.0;
    }
    int rc = check_points(bgk.data(), npts);
    if (rc != LBM_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    double* d_F = nullptr;
    rc = check_hip(hipMalloc(&d_F, sizeof(double) * 81 * (size_t)npts), "hipMalloc(F)");
    if (rc == LBM_OK) rc = jacobians(bgk.data(), npts, d_F, s);
    if (rc == LBM_OK) {
        hipLaunchKernelGGL(k_lsa_dvbe, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, s, d_F, npts, 1.0 / tau, kx,
                           ky, nk, growth);
        rc = check_hip(hipGetLastError(), "DVBE launch");
    }
    if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(s), "synchronise");
    if (d_F) (void)hipFree(d_F);
    return rc;
}

}  // extern "C"
