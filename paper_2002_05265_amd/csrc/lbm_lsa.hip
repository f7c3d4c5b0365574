// Linear stability analysis (lbm_lsa.h): the collision Jacobian J_C about a uniform flow, and the
// eigenvalues of M(k) = diag(exp(-i xi_i . k)) J_C for many wave numbers at once.
//
// J_C comes from the reverse mode of the library's own collision (lbm_adjoint_cell.hpp): with the
// adjoint seed mu = e_i, collide_adjoint returns J_C^T e_i, i.e. row i of J_C.  The eigenvalues of
// each 9 x 9 complex M(k) are found by one thread: Householder reduction to upper Hessenberg form,
// then implicit single-shift QR sweeps (Wilkinson shift from the trailing 2 x 2 block, Givens
// rotations chasing the bulge) with deflation of negligible subdiagonal entries.
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

// Eigenvalues of the 9 x 9 complex matrix H (overwritten).  Returns false if an eigenvalue did
// not converge within the iteration limit.
__device__ bool eig9(cplx (&H)[kQ][kQ], cplx (&lam)[kQ]) {
    constexpr int n = kQ;
    // Householder reduction to upper Hessenberg form: H <- P H P, P = I - 2 v v^H / |v|^2
    for (int k = 0; k < n - 2; ++k) {
        double xn2 = 0.0;
        for (int i = k + 1; i < n; ++i) xn2 += cabs2(H[i][k]);
        if (xn2 == 0.0) continue;
        const double xn = sqrt(xn2);
        const cplx x0 = H[k + 1][k];
        const double a0 = cabs(x0);
        const cplx phase = a0 > 0.0 ? cscale(x0, 1.0 / a0) : cplx{1.0, 0.0};
        const cplx alpha = cscale(phase, -xn);
        cplx v[kQ];
        for (int i = 0; i < n; ++i) v[i] = {0.0, 0.0};
        for (int i = k + 1; i < n; ++i) v[i] = H[i][k];
        v[k + 1] = csub(v[k + 1], alpha);
        double vn2 = 0.0;
        for (int i = k + 1; i < n; ++i) vn2 += cabs2(v[i]);
        if (vn2 == 0.0) continue;
        const double s = 2.0 / vn2;
        for (int j = k; j < n; ++j) {  // left: rows k+1.., w_j = v^H H[:, j]
            cplx w = {0.0, 0.0};
            for (int i = k + 1; i < n; ++i) w = cadd(w, cmul(cconj(v[i]), H[i][j]));
            w = cscale(w, s);
            for (int i = k + 1; i < n; ++i) H[i][j] = csub(H[i][j], cmul(v[i], w));
        }
        for (int i = 0; i < n; ++i) {  // right: columns k+1.., w_i = H[i, :] v
            cplx w = {0.0, 0.0};
            for (int j = k + 1; j < n; ++j) w = cadd(w, cmul(H[i][j], v[j]));
            w = cscale(w, s);
            for (int j = k + 1; j < n; ++j) H[i][j] = csub(H[i][j], cmul(w, cconj(v[j])));
        }
        for (int i = k + 2; i < n; ++i) H[i][k] = {0.0, 0.0};
    }
    double hnorm = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) hnorm = fmax(hnorm, cabs(H[i][j]));
    const double eps = 2.220446049250313e-16;
    int hi = n - 1, its = 0;
    while (hi >= 0) {
        if (hi == 0) {
            lam[0] = H[0][0];
            break;
        }
        // start l of the unreduced block ending at hi
        int l = hi;
        while (l > 0) {
            double sdiag = cabs(H[l - 1][l - 1]) + cabs(H[l][l]);
            if (sdiag == 0.0) sdiag = hnorm;
            if (cabs(H[l][l - 1]) <= 2.0 * eps * sdiag) break;
            --l;
        }
        if (l > 0) H[l][l - 1] = {0.0, 0.0};
        if (l == hi) {
            lam[hi] = H[hi][hi];
            --hi;
            its = 0;
            continue;
        }
        if (++its > 90) return false;
        // Wilkinson shift: eigenvalue of the trailing 2 x 2 block closer to H[hi][hi]
        cplx mu;
        if (its % 30 == 10 || its % 30 == 20) {  // exceptional shift
            mu = cadd(H[hi][hi], cplx{0.75 * cabs(H[hi][hi - 1]), 0.0});
        } else {
            const cplx a = H[hi - 1][hi - 1], b = H[hi - 1][hi], c = H[hi][hi - 1], d = H[hi][hi];
            const cplx half = cscale(csub(a, d), 0.5);
            const cplx disc = csqrt(cadd(cmul(half, half), cmul(b, c)));
            const cplx m1 = cadd(d, csub(half, disc)), m2 = cadd(d, cadd(half, disc));
            mu = cabs2(csub(m1, d)) <= cabs2(csub(m2, d)) ? m1 : m2;
        }
        // implicit single-shift QR sweep on rows / columns l..hi
        cplx x = csub(H[l][l], mu), y = H[l + 1][l];
        for (int k = l; k < hi; ++k) {
            const double r = sqrt(cabs2(x) + cabs2(y));
            double c;
            cplx sn;
            if (r == 0.0) {
                c = 1.0;
                sn = {0.0, 0.0};
            } else {
                const double ax = cabs(x);
                if (ax == 0.0) {
                    c = 0.0;
                    sn = cscale(cconj(y), 1.0 / cabs(y));
                } else {
                    c = ax / r;
                    sn = cscale(cmul(cscale(x, 1.0 / ax), cconj(y)), 1.0 / r);
                }
            }
            // rows k, k+1: [c s; -conj(s) c]
            for (int j = (k > l ? k - 1 : l); j <= hi; ++j) {
                const cplx a = H[k][j], b = H[k + 1][j];
                H[k][j] = cadd(cscale(a, c), cmul(sn, b));
                H[k + 1][j] = csub(cscale(b, c), cmul(cconj(sn), a));
            }
            // columns k, k+1 (similarity with the conjugate transpose)
            const int iend = k + 2 < hi ? k + 2 : hi;
            for (int i = l; i <= iend; ++i) {
                const cplx a = H[i][k], b = H[i][k + 1];
                H[i][k] = cadd(cscale(a, c), cmul(b, cconj(sn)));
                H[i][k + 1] = csub(cscale(b, c), cmul(a, sn));
            }
            if (k < hi - 1) {
                x = H[k + 1][k];
                y = H[k + 2][k];
            }
        }
    }
    return true;
}

// M(k) = diag(exp(-i xi . k)) J for wave number (kx, ky).
__device__ void build_m(const double* __restrict__ J, double kx, double ky, cplx (&H)[kQ][kQ]) {
    for (int i = 0; i < kQ; ++i) {
        double sn, cs;
        sincos(-((double)cx(i) * kx + (double)cy(i) * ky), &sn, &cs);
        for (int j = 0; j < kQ; ++j) {
            const double v = J[i * 9 + j];
            H[i][j] = {cs * v, sn * v};
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
    for (int m = 0; m < kQ; ++m) {
        out[((size_t)q * kQ + m) * 2] = ok ? lam[m].re : NAN;
        out[((size_t)q * kQ + m) * 2 + 1] = ok ? lam[m].im : NAN;
    }
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

}  // extern "C"
