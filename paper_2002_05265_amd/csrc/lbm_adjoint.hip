// Discrete adjoint kernels (include/lbm_adjoint.h).
//
// One reverse step reads f_n (pull from the raw state, exactly as the forward step does),
// lambda_{n+1} at x + xi_i (transpose of the streaming permutation) and writes lambda_n at x:
// 27 stored values per node, no atomics.  Two reverse steps in one launch keep lambda_n in LDS:
// 36 stored values per node and pair.  The rate gradients are reduced per strip in FP64,
// accumulated per strip over the steps of a sweep, and summed into the caller's accumulator in a
// fixed order at the end.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "lbm.h"
#include "lbm_adjoint.h"
#include "lbm_adjoint_cell.hpp"
#include "lbm_cell.hpp"
#include "lbm_internal.hpp"

using namespace lbm;

namespace {

// Every reverse step walks the grid in strips of 64 columns and AdjShape::hs rows, one
// workgroup of kAdjWaves waves per strip (lane l takes column x0 + l), and the strip is the unit
// of the rate-gradient sums: the workgroup of block b adds its strip's FP64 sum to slot b.  Wave w
// takes rows ys + w, ys + w + kAdjWaves, ... of its strip in increasing order, in the one-step
// and the two-step kernel alike, so both add up every step's terms of a slot in the same order and
// the gradients do not depend on which reverse steps were paired in one launch.
#ifndef LBM_ADJ_WAVES
#define LBM_ADJ_WAVES 4
#endif
#ifndef LBM_ADJ_UNROLL
#define LBM_ADJ_UNROLL 1
#endif
#ifndef LBM_ADJ_STRIPS
#define LBM_ADJ_STRIPS 2048
#endif
#ifndef LBM_ADJ_MAX_ROWS
#define LBM_ADJ_MAX_ROWS 64
#endif
#ifndef LBM_ADJ_XCD
#define LBM_ADJ_XCD 0
#endif
#ifndef LBM_ADJ_GROUP
#define LBM_ADJ_GROUP 16
#endif
constexpr int kAdjWaves = LBM_ADJ_WAVES;
constexpr int kAdjRing = 8;  // rows per pass of the two-step kernel (a multiple of kAdjWaves)
constexpr int kAdjUnroll = LBM_ADJ_UNROLL;  // rows per wave and iteration of the one-step kernel

struct AdjShape {
    int hs;           // strip rows, a multiple of kAdjRing
    unsigned sx, nb;  // strips across, strips in all
};

AdjShape adjoint_shape(const lbm_ctx* ctx) {
    AdjShape a;
    a.sx = (unsigned)((ctx->nx + 63) / 64);
    // about LBM_ADJ_STRIPS strips where the grid has them, 8 to LBM_ADJ_MAX_ROWS rows each
    const long long target = (long long)ctx->ny * a.sx / LBM_ADJ_STRIPS;
    const long long h = (target + kAdjRing / 2) / kAdjRing * kAdjRing;
    a.hs = (int)(h < kAdjRing ? kAdjRing : (h > LBM_ADJ_MAX_ROWS ? LBM_ADJ_MAX_ROWS : h));
    a.nb = a.sx * (unsigned)((ctx->ny + a.hs - 1) / a.hs);
    return a;
}

unsigned adjoint_blocks(const lbm_ctx* ctx) { return adjoint_shape(ctx).nb; }

// Strip (bx, by) of block b: in FP32 and FP16 by groups of LBM_ADJ_GROUP strip columns
// (strip_of_block_grouped), so that neighbouring strips share their edge lines in one L2.  Measured at
// 4096^2: FP32 two reverse steps per launch 5% faster with G = 16 than in hardware order (G = 8:
// 4%; 4 and 2: 12-24% slower), FP64 2-6% slower, so FP64 keeps the hardware order (G = 0, or
// tile_of_block's bands when xcd is set).
template <int PREC>
__device__ __forceinline__ void strip_of_block(unsigned b, unsigned sx, unsigned nb, int xcd, unsigned& bx,
                                               unsigned& by) {
    if constexpr (PREC != kF64 && LBM_ADJ_GROUP > 0) {
        strip_of_block_grouped(b, sx, nb, LBM_ADJ_GROUP, bx, by);
    } else {
        tile_of_block(b, sx, nb, xcd, bx, by);
    }
}

template <int PREC> struct AdjT;
template <> struct AdjT<kF64> { using T = double; };
template <> struct AdjT<kF32> { using T = float; };
template <> struct AdjT<kF16> { using T = float; };

// mu_i(x) = lam_i(x + xi_i)
template <typename T, typename R>
__device__ __forceinline__ void push_gather(const T* __restrict__ lam, long long plane, const Nbr& n,
                                            R (&mu)[9]) {
    constexpr unsigned E = sizeof(T);
    const unsigned r0 = n.r0 * E, rm = n.rm * E, rp = n.rp * E;
    const unsigned x0 = n.x * E, xm = n.xm * E, xp = n.xp * E;
    mu[0] = R(*plane_at(lam, plane, 0, r0 + x0));
    mu[1] = R(*plane_at(lam, plane, 1, r0 + xp));
    mu[2] = R(*plane_at(lam, plane, 2, rp + x0));
    mu[3] = R(*plane_at(lam, plane, 3, r0 + xm));
    mu[4] = R(*plane_at(lam, plane, 4, rm + x0));
    mu[5] = R(*plane_at(lam, plane, 5, rp + xp));
    mu[6] = R(*plane_at(lam, plane, 6, rp + xm));
    mu[7] = R(*plane_at(lam, plane, 7, rm + xm));
    mu[8] = R(*plane_at(lam, plane, 8, rm + xp));
}

// Rate-gradient slots: block b adds (accumulate = 1) or writes (0) its strip's FP64 sums to slot
// b, the first reverse step's before the second's (two reverse steps per launch: a, then b), as
// two one-step launches would.  A slot is touched by one block per launch and launches are
// stream-ordered, so no atomics or fences are needed; one k_finalize_add per host call folds the
// slots into domega.
template <bool TWO>
__device__ __forceinline__ void slots_add(double (&a)[5], double (&b)[5], double* __restrict__ slots,
                                          int accumulate) {
    __shared__ double ta[5], tb[5];
    block_sum<5>(a, ta);
    __syncthreads();
    if constexpr (TWO) {
        block_sum<5>(b, tb);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* p = slots + 5 * (size_t)blockIdx.x;
        for (int k = 0; k < 5; ++k) {
            double v = (accumulate ? p[k] : 0.0) + ta[k];
            if constexpr (TWO) v += tb[k];
            p[k] = v;
        }
    }
}

// out[k] += sum over blocks of slots[5 b + k] (one block, fixed order).
__global__ __launch_bounds__(256) void k_finalize_add(const double* __restrict__ slots, int nblocks,
                                                      double* __restrict__ out) {
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int k = 0; k < 5; ++k) v[k] += slots[5 * (size_t)b + k];
    __shared__ double tot[5];
    block_sum<5>(v, tot);
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) out[k] += tot[k];
}

// One node of a reverse step: hb = lambda_n(x, y) = J_C(h)^T mu for the pulled state h of f_n and
// mu_i = lambda_{n+1}(x + xi_i); when `count`, the node's rate-gradient terms are added to ws.
template <int MODEL, int PREC>
__device__ __forceinline__ void reverse_core(const typename Store<PREC>::R (&h)[9],
                                             const typename Store<PREC>::R (&mu)[9],
                                             const Coef<typename Store<PREC>::R>& c,
                                             const Ref<typename Store<PREC>::R>& ref, int N,
                                             typename Store<PREC>::R (&hb)[9], double (&ws)[5], bool count) {
    using R = typename Store<PREC>::R;
    double rho_d;
    const Macro<R> m = macro_of<typename Store<PREC>::S>(h, ref, rho_d);
    R cb[7] = {R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
    collide_adjoint<MODEL>(h, m, ref, c, N, mu, hb, cb);
    if (count) {
        double wn[5];
        omega_adjoint(cb, wn);
#pragma unroll
        for (int k = 0; k < 5; ++k) ws[k] += wn[k];
    }
}

// The same node with f_n pulled from `state` and mu gathered from lam_next in memory.
template <int MODEL, int PREC>
__device__ __forceinline__ void reverse_node(const typename Store<PREC>::S* __restrict__ state,
                                             const typename AdjT<PREC>::T* __restrict__ lam_next, const Geom& g,
                                             int x, int y, const Coef<typename Store<PREC>::R>& c,
                                             const Ref<typename Store<PREC>::R>& ref, int N,
                                             typename Store<PREC>::R (&hb)[9], double (&ws)[5], bool count) {
    using R = typename Store<PREC>::R;
    const Nbr n = neighbours(x, y, g.nx, g.ny);
    R h[9], mu[9];
    pull_load(state, g.plane, n, h);
    push_gather(lam_next, g.plane, n, mu);
    reverse_core<MODEL, PREC>(h, mu, c, ref, N, hb, ws, count);
}

template <typename T, typename R>
__device__ __forceinline__ void store_lam(T* __restrict__ lam, const Geom& g, int x, int y, const R (&hb)[9]) {
    // lambda is read back only by the next reverse step, as a gather over the whole grid:
    // streaming stores keep it from displacing reusable lines
    const unsigned o = ((unsigned)y * (unsigned)g.nx + (unsigned)x) * (unsigned)sizeof(T);
#pragma unroll
    for (int i = 0; i < 9; ++i) st<T>(plane_at(lam, g.plane, i, o), T(hb[i]));
}

// One reverse step (lambda_{n+1} -> lambda_n at state f_n) over one strip per workgroup.
template <int MODEL, int PREC>
__global__ __launch_bounds__(64 * kAdjWaves) void k_adjoint_strip1(
    const typename Store<PREC>::S* __restrict__ state, const typename AdjT<PREC>::T* __restrict__ lam_next,
    typename AdjT<PREC>::T* __restrict__ lam, Geom g, Coef<typename Store<PREC>::R> c,
    Ref<typename Store<PREC>::R> ref, int N, double* __restrict__ slots, int accumulate, int hs, unsigned sx,
    unsigned nb, int xcd) {
    using R = typename Store<PREC>::R;
    unsigned bx, by;
    strip_of_block<PREC>(blockIdx.x, sx, nb, xcd, bx, by);
    const int x = (int)bx * 64 + (int)(threadIdx.x & 63u);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ys = (int)by * hs, ye = min(ys + hs, g.ny);
    double ws[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (x < g.nx) {
        for (int yb = ys + wave; yb < ye; yb += kAdjWaves * kAdjUnroll) {
#pragma unroll
            for (int u = 0; u < kAdjUnroll; ++u) {
                const int y = yb + u * kAdjWaves;
                if (y < ye) {
                    R hb[9];
                    reverse_node<MODEL, PREC>(state, lam_next, g, x, y, c, ref, N, hb, ws, true);
                    store_lam(lam, g, x, y, hb);
                }
            }
        }
    }
    slots_add<false>(ws, ws, slots, accumulate);
}

// Two reverse steps per pass over one strip per workgroup: lambda_{n+1} -> lambda_n at f_n (the
// first, on the strip plus one halo row and column on each side, kept in an LDS ring of
// kAdjRing + 2 rows of 66 columns) -> lambda_{n-1} at f_{n-1} (the second, gathered from the
// ring, written to memory).  lambda_n never goes to memory: per node and pair of steps the
// launch reads f_n, f_{n-1} and lambda_{n+1} and writes lambda_{n-1}, 18 s + 18 a bytes against
// 2 (9 s + 18 a) for two one-step launches.  A pass computes the first step on rows yb + 1 ..
// yb + kAdjRing and the second on rows yb .. yb + kAdjRing - 1, with a barrier after each.  The
// ring holds the adjoint type, as memory would, and every node runs the arithmetic of
// k_adjoint_strip1, so lambda_{n-1} and the gradient sums are bit-identical to two one-step
// launches.  Wave kAdjWaves - 1 also takes the halo columns (two lanes per row).
template <int MODEL, int PREC>
__global__ __launch_bounds__(64 * kAdjWaves) void k_adjoint_strip2(
    const typename Store<PREC>::S* __restrict__ state_n, const typename Store<PREC>::S* __restrict__ state_m,
    const typename AdjT<PREC>::T* __restrict__ lam_next, typename AdjT<PREC>::T* __restrict__ lam, Geom g,
    Coef<typename Store<PREC>::R> c, Ref<typename Store<PREC>::R> ref, int N, double* __restrict__ slots,
    int accumulate, int hs, unsigned sx, unsigned nb, int xcd) {
    using R = typename Store<PREC>::R;
    using T = typename AdjT<PREC>::T;
    constexpr int NR = kAdjRing + 2;
    constexpr int KR = kAdjRing / kAdjWaves;
    static_assert(kAdjRing % kAdjWaves == 0 && 2 * kAdjRing <= 64, "ring rows");
    __shared__ T ring[9][NR][66];
    unsigned bx, by;
    strip_of_block<PREC>(blockIdx.x, sx, nb, xcd, bx, by);
    const int x0 = (int)bx * 64;
    const int lane = (int)(threadIdx.x & 63u);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ys = (int)by * hs, ye = min(ys + hs, g.ny);
    const int w = min(64, g.nx - x0);
    const bool in = lane < w;
    const int x = x0 + lane;
    // ring column 0 holds grid column x0 - 1, column 1 + l column x0 + l, column w + 1 x0 + w
    const int xl = x0 == 0 ? g.nx - 1 : x0 - 1;
    const int xr = x0 + w == g.nx ? 0 : x0 + w;
    double wa[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, wb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // first step at grid column xg and strip row r (ys - 1 <= r <= ye, wrapped here) into ring
    // column cc
    auto first = [&](int xg, int r, int cc, bool count) {
        R hb[9];
        const int yw = r < 0 ? r + g.ny : (r >= g.ny ? r - g.ny : r);
        reverse_node<MODEL, PREC>(state_n, lam_next, g, xg, yw, c, ref, N, hb, wa, count);
        const int s = (r - ys + 1) % NR;
#pragma unroll
        for (int i = 0; i < 9; ++i) ring[i][s][cc] = T(hb[i]);
    };
    // the halo columns of rows r0 .. r1
    auto halo = [&](int r0, int r1) {
        if (wave == kAdjWaves - 1) {
            const int r = r0 + (lane >> 1);
            if (lane < 2 * kAdjRing && r <= r1) first((lane & 1) ? xr : xl, r, (lane & 1) ? w + 1 : 0, false);
        }
    };
    // prologue: rows ys - 1 (halo) and ys (wave 0's first row)
    if (in) {
        if (wave == 0)
            first(x, ys, lane + 1, true);
        else if (wave == 1)
            first(x, ys - 1, lane + 1, false);
    }
    halo(ys - 1, ys);
    __syncthreads();
    // wave w's first-step rows in a pass: yb + m0 + kAdjWaves k (the rows w mod kAdjWaves from ys)
    const int m0 = (wave + kAdjWaves - 1) % kAdjWaves + 1;
    for (int yb = ys; yb < ye; yb += kAdjRing) {
        const int top = min(yb + kAdjRing, ye);  // first step: rows yb + 1 .. top (row ye: halo)
        if (in) {
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const int r = yb + m0 + kAdjWaves * k;
                if (r <= top) first(x, r, lane + 1, r < ye);
            }
        }
        halo(yb + 1, top);
        __syncthreads();
        if (in) {
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const int y = yb + wave + kAdjWaves * k;
                if (y < ye) {
                    const int s0 = y - ys + 1;  // ring slot of row y, before wrapping
                    R h[9], mu[9], hb[9];
#pragma unroll
                    for (int i = 0; i < 9; ++i) mu[i] = R(ring[i][(s0 + cy(i)) % NR][lane + 1 + cx(i)]);
                    pull_load(state_m, g.plane, neighbours(x, y, g.nx, g.ny), h);
                    reverse_core<MODEL, PREC>(h, mu, c, ref, N, hb, wb, true);
                    store_lam(lam, g, x, y, hb);
                }
            }
        }
        __syncthreads();
    }
    slots_add<true>(wa, wb, slots, accumulate);
}

// Velocity of the current state in FP64 (pull).
template <int PREC>
__device__ __forceinline__ void node_velocity(const typename Store<PREC>::S* __restrict__ src, const Geom& g,
                                              const Nbr& nb, const Ref<double>& ref, double& rho,
                                              double& u, double& v) {
    double h[9];
    pull_load(src, g.plane, nb, h);
    rho = ref.rho + (((h[0] + (h[1] + h[3])) + (h[2] + h[4])) + ((h[5] + h[7]) + (h[6] + h[8])));
    const double jx = ((h[1] + h[5] + h[8]) - (h[3] + h[6] + h[7])) + ref.rho * ref.ux;
    const double jy = ((h[2] + h[5] + h[6]) - (h[4] + h[7] + h[8])) + ref.rho * ref.uy;
    u = jx / rho;
    v = jy / rho;
}

template <int PREC>
__global__ __launch_bounds__(256) void k_loss_l2(const typename Store<PREC>::S* __restrict__ src, Geom g,
                                                 Ref<double> ref, const double* __restrict__ ux_t,
                                                 const double* __restrict__ uy_t,
                                                 double* __restrict__ partials) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (x < g.nx && y < g.ny) {
        const Nbr nb = neighbours(x, y, g.nx, g.ny);
        double rho, u, w;
        node_velocity<PREC>(src, g, nb, ref, rho, u, w);
        const unsigned c = nb.r0 + (unsigned)x;
        const double ex = u - ux_t[c], ey = w - uy_t[c];
        v[0] = ex * ex + ey * ey;
    }
    block_sum<5>(v, partials + 5 * (size_t)(blockIdx.y * gridDim.x + blockIdx.x));
}

// lam_i = (1 / L) sum_a (u_a - t_a) (xi_ia - u_a) / rho
template <int PREC>
__global__ __launch_bounds__(256) void k_seed_l2(const typename Store<PREC>::S* __restrict__ src, Geom g,
                                                 Ref<double> ref, const double* __restrict__ ux_t,
                                                 const double* __restrict__ uy_t, double inv_loss,
                                                 typename AdjT<PREC>::T* __restrict__ lam) {
    using T = typename AdjT<PREC>::T;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= g.nx || y >= g.ny) return;
    const Nbr nb = neighbours(x, y, g.nx, g.ny);
    double rho, u, w;
    node_velocity<PREC>(src, g, nb, ref, rho, u, w);
    const unsigned c = nb.r0 + (unsigned)x;
    const double gx = (u - ux_t[c]) * inv_loss / rho, gy = (w - uy_t[c]) * inv_loss / rho;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        lam[i * g.plane + c] = T(gx * ((double)cx(i) - u) + gy * ((double)cy(i) - w));
}

// dL/du0 through f_0 = f^eq_N(rho0, u0) (reverse of eq_deviation in FP64).
template <int PREC>
__global__ __launch_bounds__(256) void k_eq_vjp(Geom g, Ref<double> ref, int N, const double* __restrict__ rho0,
                                                const double* __restrict__ ux0, const double* __restrict__ uy0,
                                                const typename AdjT<PREC>::T* __restrict__ lam0,
                                                double* __restrict__ dux, double* __restrict__ duy) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= g.nx || y >= g.ny) return;
    const unsigned c = (unsigned)y * (unsigned)g.nx + (unsigned)x;
    const Macro<double> m = macro_of_fields(rho0[c], ux0[c], uy0[c], ref);
    double mu[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) mu[i] = (double)lam0[i * g.plane + c];
    MacroBar<double> mb;
    zero(mb);
    double ab[6];
    pop_adjoint(mu, mb, ab);
    eq_adjoint(m, ref, N, ab, mb);
    // dux = ux - Ux, jx = rho ux - rho_s Ux
    dux[c] = mb.ux + mb.dux + m.rho * mb.jx;
    duy[c] = mb.uy + mb.duy + m.rho * mb.jy;
}

// One reverse step (state_m == NULL: lambda_{n+1} = lam_next -> lambda_n = lam at f_n = state_n)
// or two (lam_next -> lambda_{n-1} = lam through f_n = state_n and f_{n-1} = state_m).
template <int MODEL, int PREC>
void launch_adj_t(lbm_ctx* ctx, const double* w, const void* state_n, const void* state_m, const void* lam_next,
                  void* lam, int accumulate) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    using T = typename AdjT<PREC>::T;
    const AdjShape a = adjoint_shape(ctx);
    if (state_m)
        hipLaunchKernelGGL((k_adjoint_strip2<MODEL, PREC>), dim3(a.nb), dim3(64 * kAdjWaves), 0, ctx->stream,
                           reinterpret_cast<const S*>(state_n), reinterpret_cast<const S*>(state_m),
                           reinterpret_cast<const T*>(lam_next), reinterpret_cast<T*>(lam), ctx->geom(),
                           make_coef<R>(w), ref_as<R>(ctx->ref), ctx->eq_order, ctx->d_wslots, accumulate, a.hs,
                           a.sx, a.nb, LBM_ADJ_XCD);
    else
        hipLaunchKernelGGL((k_adjoint_strip1<MODEL, PREC>), dim3(a.nb), dim3(64 * kAdjWaves), 0, ctx->stream,
                           reinterpret_cast<const S*>(state_n), reinterpret_cast<const T*>(lam_next),
                           reinterpret_cast<T*>(lam), ctx->geom(), make_coef<R>(w), ref_as<R>(ctx->ref),
                           ctx->eq_order, ctx->d_wslots, accumulate, a.hs, a.sx, a.nb, LBM_ADJ_XCD);
}

template <int PREC>
void launch_adj_p(lbm_ctx* ctx, int model, const double* w, const void* sn, const void* sm, const void* lam_next,
                  void* lam, int acc) {
    switch (model) {
        case LBM_BGK: launch_adj_t<kBGK, PREC>(ctx, w, sn, sm, lam_next, lam, acc); break;
        case LBM_RM: launch_adj_t<kRM, PREC>(ctx, w, sn, sm, lam_next, lam, acc); break;
        case LBM_HM: launch_adj_t<kHM, PREC>(ctx, w, sn, sm, lam_next, lam, acc); break;
        case LBM_CM: launch_adj_t<kCM, PREC>(ctx, w, sn, sm, lam_next, lam, acc); break;
        case LBM_CHM: launch_adj_t<kCHM, PREC>(ctx, w, sn, sm, lam_next, lam, acc); break;
        case LBM_K: launch_adj_t<kK, PREC>(ctx, w, sn, sm, lam_next, lam, acc); break;
        case LBM_PR: launch_adj_t<kPR, PREC>(ctx, w, sn, sm, lam_next, lam, acc); break;
        case LBM_RR: launch_adj_t<kRR, PREC>(ctx, w, sn, sm, lam_next, lam, acc); break;
        default: launch_adj_t<kStreamOnly, PREC>(ctx, w, sn, sm, lam_next, lam, acc); break;
    }
}

size_t adj_elem(int prec) { return prec == LBM_F64 ? 8 : 4; }

}  // namespace

extern "C" {

size_t lbm_state_bytes(lbm_ctx* ctx) { return ctx ? (size_t)9 * (size_t)ctx->plane * ctx->esize : 0; }

size_t lbm_adjoint_bytes(lbm_ctx* ctx) {
    return ctx ? (size_t)9 * (size_t)ctx->plane * adj_elem(ctx->prec) : 0;
}

int lbm_save_state(lbm_ctx* ctx, void* dst) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (!dst) return set_error(LBM_EINVAL, "dst is NULL");
    return check_hip(hipMemcpyAsync(dst, ctx->copy(ctx->cur), lbm_state_bytes(ctx), hipMemcpyDeviceToDevice,
                                    ctx->stream),
                     "save state");
}

int lbm_load_state(lbm_ctx* ctx, const void* src, long long step) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (!src) return set_error(LBM_EINVAL, "src is NULL");
    if (step < 0 || step >= INT_MAX) return set_error(LBM_EINVAL, "step %lld out of range", step);
    int rc = check_hip(hipMemcpyAsync(ctx->copy(ctx->cur), src, lbm_state_bytes(ctx), hipMemcpyDeviceToDevice,
                                      ctx->stream),
                       "load state");
    if (rc != LBM_OK) return rc;
    ctx->step = step;
    return reset_blowup(ctx);
}

int lbm_adjoint_seed_velocity_l2(lbm_ctx* ctx, const double* ux_t, const double* uy_t, void* lam,
                                 double* loss) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (!ux_t || !uy_t || !lam || !loss) return set_error(LBM_EINVAL, "NULL pointer");
    const Launch l = launch_for(ctx->nx, ctx->ny);
    const char* src = ctx->copy(ctx->cur);
    switch (ctx->prec) {
        case LBM_F64:
            hipLaunchKernelGGL(k_loss_l2<kF64>, l.grid, l.block, 0, ctx->stream, reinterpret_cast<const double*>(src),
                               ctx->geom(), ctx->ref, ux_t, uy_t, ctx->d_part);
            break;
        case LBM_F32_SHIFTED:
            hipLaunchKernelGGL(k_loss_l2<kF32>, l.grid, l.block, 0, ctx->stream, reinterpret_cast<const float*>(src),
                               ctx->geom(), ctx->ref, ux_t, uy_t, ctx->d_part);
            break;
        default:
            hipLaunchKernelGGL(k_loss_l2<kF16>, l.grid, l.block, 0, ctx->stream,
                               reinterpret_cast<const _Float16*>(src), ctx->geom(), ctx->ref, ux_t, uy_t, ctx->d_part);
            break;
    }
    int rc = check_hip(hipGetLastError(), "loss kernel launch");
    if (rc != LBM_OK) return rc;
    rc = reduce_partials(ctx);
    double t[5];
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpyAsync(t, ctx->d_tot, sizeof(t), hipMemcpyDeviceToHost, ctx->stream), "copy loss");
    if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(ctx->stream), "synchronise");
    if (rc != LBM_OK) return rc;
    const double L = std::sqrt(t[0]);
    *loss = L;
    if (!(L > 0.0)) return set_error(LBM_EINVAL, "loss is %g: the seed 1/L is undefined", L);
    switch (ctx->prec) {
        case LBM_F64:
            hipLaunchKernelGGL(k_seed_l2<kF64>, l.grid, l.block, 0, ctx->stream, reinterpret_cast<const double*>(src),
                               ctx->geom(), ctx->ref, ux_t, uy_t, 1.0 / L, reinterpret_cast<double*>(lam));
            break;
        case LBM_F32_SHIFTED:
            hipLaunchKernelGGL(k_seed_l2<kF32>, l.grid, l.block, 0, ctx->stream, reinterpret_cast<const float*>(src),
                               ctx->geom(), ctx->ref, ux_t, uy_t, 1.0 / L, reinterpret_cast<float*>(lam));
            break;
        default:
            hipLaunchKernelGGL(k_seed_l2<kF16>, l.grid, l.block, 0, ctx->stream,
                               reinterpret_cast<const _Float16*>(src), ctx->geom(), ctx->ref, ux_t, uy_t, 1.0 / L,
                               reinterpret_cast<float*>(lam));
            break;
    }
    return check_hip(hipGetLastError(), "seed kernel launch");
}

int lbm_adjoint_step(lbm_ctx* ctx, int model, const double* omega, const void* state,
                     const void* lam_next, void* lam, double* domega) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (!lam_next || !lam || !domega) return set_error(LBM_EINVAL, "NULL pointer");
    const void* st = state ? state : ctx->copy(ctx->cur);
    void* lams[2] = {const_cast<void*>(lam_next), lam};
    return lbm_adjoint_many(ctx, model, omega, &st, 1, lams, domega);
}

int lbm_adjoint_many(lbm_ctx* ctx, int model, const double* omega, const void* const* states,
                     int count, void* const* lam, double* domega) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (count < 0) return set_error(LBM_EINVAL, "count %d < 0", count);
    if (count > 0 && (!states || !lam)) return set_error(LBM_EINVAL, "NULL pointer array");
    for (int k = 0; k < count; ++k)
        if (!states[k] || !lam[k] || !lam[k + 1] || lam[k] == lam[k + 1])
            return set_error(LBM_EINVAL, "bad pointer at reverse step %d", k);
    int rc = validate_model(model, ctx->eq_order);
    if (rc == LBM_OK) rc = validate_omega(omega);
    if (rc != LBM_OK) return rc;
    if (!ctx->d_wslots) {
        rc = check_hip(hipMalloc(&ctx->d_wslots, sizeof(double) * 5 * (size_t)adjoint_blocks(ctx)), "hipMalloc(slots)");
        if (rc != LBM_OK) return rc;
    }
    for (int k = 0; k < count;) {
        const int acc = ctx->wslots_live ? 1 : 0;
        // two reverse steps in one launch when the context asks for it and the pair's output
        // buffer is not its input (other workgroups still gather lambda_{n+1} around their strips
        // while one writes lambda_{n-1}); lam[k + 1] is then not written
        const bool pair = ctx->adj_depth == 2 && k + 1 < count && lam[k + 2] != lam[k];
        const void* sm = pair ? states[k + 1] : nullptr;
        void* out = pair ? lam[k + 2] : lam[k + 1];
        switch (ctx->prec) {
            case LBM_F64: launch_adj_p<kF64>(ctx, model, omega, states[k], sm, lam[k], out, acc); break;
            case LBM_F32_SHIFTED: launch_adj_p<kF32>(ctx, model, omega, states[k], sm, lam[k], out, acc); break;
            default: launch_adj_p<kF16>(ctx, model, omega, states[k], sm, lam[k], out, acc); break;
        }
        ctx->wslots_live = true;
        k += pair ? 2 : 1;
    }
    rc = check_hip(hipGetLastError(), "adjoint kernel launch");
    if (rc != LBM_OK || !domega) return rc;
    return lbm_adjoint_flush(ctx, domega);
}

int lbm_set_adjoint_depth(lbm_ctx* ctx, int steps) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (steps != 1 && steps != 2) return set_error(LBM_EINVAL, "reverse steps per launch %d not in {1, 2}", steps);
    ctx->adj_depth = steps;
    return LBM_OK;
}

int lbm_get_adjoint_depth(lbm_ctx* ctx, int* steps) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (steps) *steps = ctx->adj_depth;
    return LBM_OK;
}

int lbm_adjoint_flush(lbm_ctx* ctx, double* domega) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (!domega) return set_error(LBM_EINVAL, "domega is NULL");
    if (!ctx->wslots_live) return LBM_OK;
    hipLaunchKernelGGL(k_finalize_add, dim3(1), dim3(256), 0, ctx->stream, ctx->d_wslots,
                       (int)adjoint_blocks(ctx), domega);
    ctx->wslots_live = false;
    return check_hip(hipGetLastError(), "adjoint reduction launch");
}

int lbm_eq_vjp(lbm_ctx* ctx, const double* rho0, const double* ux0, const double* uy0,
               const void* lam0, double* dux, double* duy) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (!rho0 || !ux0 || !uy0 || !lam0 || !dux || !duy) return set_error(LBM_EINVAL, "NULL pointer");
    const Launch l = launch_for(ctx->nx, ctx->ny);
    if (ctx->prec == LBM_F64)
        hipLaunchKernelGGL(k_eq_vjp<kF64>, l.grid, l.block, 0, ctx->stream, ctx->geom(), ctx->ref, ctx->eq_order,
                           rho0, ux0, uy0, reinterpret_cast<const double*>(lam0), dux, duy);
    else
        hipLaunchKernelGGL(k_eq_vjp<kF32>, l.grid, l.block, 0, ctx->stream, ctx->geom(), ctx->ref, ctx->eq_order,
                           rho0, ux0, uy0, reinterpret_cast<const float*>(lam0), dux, duy);
    return check_hip(hipGetLastError(), "eq_vjp kernel launch");
}

}  // extern "C"
