// Discrete adjoint kernels (include/lbm_adjoint.h).
//
// One reverse step reads f_n (pull from the raw state, exactly as the forward step does),
// lambda_{n+1} at x + xi_i (transpose of the streaming permutation) and writes lambda_n at x:
// 27 stored values per node, no atomics.  The rate gradients are reduced per block in FP64,
// accumulated per block over the steps of one call, and summed into the caller's accumulator
// in a fixed order at the end of the call.
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

// Every reverse step of a context uses this one launch shape, so the launches that feed one set
// of rate-gradient slots (block b writes slot b) have the same blocks.  Two nodes per thread
// halve the per-block gradient reductions; at 4096^2 that is 4-7% faster with 4-byte adjoint
// values and 2% slower with 8-byte ones (one node per thread there).
StepShape adjoint_shape(const lbm_ctx* ctx) {
    return step_shape(ctx->nx, ctx->ny, ctx->prec == LBM_F64 ? 1 : 2, LBM_DEFAULT_XCD);
}

unsigned adjoint_blocks(const lbm_ctx* ctx) {
    const StepShape sh = adjoint_shape(ctx);
    return sh.gx * sh.gy;
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

// Per-block rate-gradient slots: block b adds (accumulate = 1) or writes (0) its FP64 block sum
// to slot b.  A slot is touched by one block per launch and launches are stream-ordered, so no
// atomics or fences are needed; one k_finalize_add per host call folds the slots into domega.
__device__ __forceinline__ void block_accumulate(double (&v)[5], double* __restrict__ slots, int accumulate) {
    __shared__ double tot[5];
    block_sum<5>(v, tot);
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double* p = slots + 5 * (size_t)blockIdx.x;
        for (int k = 0; k < 5; ++k) p[k] = (accumulate ? p[k] : 0.0) + tot[k];
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

template <int MODEL, int PREC, int ROWS>
__global__ __launch_bounds__(256) void k_adjoint_step(const typename Store<PREC>::S* __restrict__ state,
                                                      const typename AdjT<PREC>::T* __restrict__ lam_next,
                                                      typename AdjT<PREC>::T* __restrict__ lam, Geom g,
                                                      Coef<typename Store<PREC>::R> c,
                                                      Ref<typename Store<PREC>::R> ref, int N,
                                                      double* __restrict__ slots, int accumulate,
                                                      unsigned gx, unsigned nb, int xcd) {
    using R = typename Store<PREC>::R;
    using T = typename AdjT<PREC>::T;
    unsigned bx, by;
    tile_of_block(blockIdx.x, gx, nb, xcd, bx, by);
    const int x = bx * blockDim.x + threadIdx.x;
    const int y0 = by * blockDim.y * ROWS + threadIdx.y;
    double wb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (x < g.nx) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int y = y0 + r * (int)blockDim.y;
            if (y < g.ny) {
                const Nbr n = neighbours(x, y, g.nx, g.ny);
                R h[9], mu[9], hb[9];
                pull_load(state, g.plane, n, h);
                push_gather(lam_next, g.plane, n, mu);
                double rho_d;
                const Macro<R> m = macro_of<typename Store<PREC>::S>(h, ref, rho_d);
                R cb[7] = {R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
                collide_adjoint<MODEL>(h, m, ref, c, N, mu, hb, cb);
                const unsigned o = (n.r0 + (unsigned)x) * (unsigned)sizeof(T);
                // lambda_n is read back only by the next reverse step, as a gather over the
                // whole grid: streaming stores keep it from displacing reusable lines
#pragma unroll
                for (int i = 0; i < 9; ++i) st<T>(plane_at(lam, g.plane, i, o), T(hb[i]));
                double wn[5];
                omega_adjoint(cb, wn);
#pragma unroll
                for (int k = 0; k < 5; ++k) wb[k] += wn[k];
            }
        }
    }
    block_accumulate(wb, slots, accumulate);
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

template <int MODEL, int PREC, int ROWS>
void launch_adj_r(lbm_ctx* ctx, const StepShape& sh, const double* w, const void* state, const void* lam_next,
                  void* lam, int accumulate) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    using T = typename AdjT<PREC>::T;
    const unsigned nb = sh.gx * sh.gy;
    hipLaunchKernelGGL((k_adjoint_step<MODEL, PREC, ROWS>), dim3(nb), dim3(sh.bw, sh.bh), 0, ctx->stream,
                       reinterpret_cast<const S*>(state), reinterpret_cast<const T*>(lam_next),
                       reinterpret_cast<T*>(lam), ctx->geom(), make_coef<R>(w), ref_as<R>(ctx->ref),
                       ctx->eq_order, ctx->d_wslots, accumulate, sh.gx, nb, sh.xcd);
}

template <int MODEL, int PREC>
void launch_adj_t(lbm_ctx* ctx, const double* w, const void* state, const void* lam_next, void* lam,
                  int accumulate) {
    const StepShape sh = adjoint_shape(ctx);
    if (sh.rows == 2)
        launch_adj_r<MODEL, PREC, 2>(ctx, sh, w, state, lam_next, lam, accumulate);
    else
        launch_adj_r<MODEL, PREC, 1>(ctx, sh, w, state, lam_next, lam, accumulate);
}

template <int PREC>
void launch_adj_p(lbm_ctx* ctx, int model, const double* w, const void* state, const void* lam_next,
                  void* lam, int accumulate) {
    switch (model) {
        case LBM_BGK: launch_adj_t<kBGK, PREC>(ctx, w, state, lam_next, lam, accumulate); break;
        case LBM_RM: launch_adj_t<kRM, PREC>(ctx, w, state, lam_next, lam, accumulate); break;
        case LBM_HM: launch_adj_t<kHM, PREC>(ctx, w, state, lam_next, lam, accumulate); break;
        case LBM_CM: launch_adj_t<kCM, PREC>(ctx, w, state, lam_next, lam, accumulate); break;
        case LBM_CHM: launch_adj_t<kCHM, PREC>(ctx, w, state, lam_next, lam, accumulate); break;
        case LBM_K: launch_adj_t<kK, PREC>(ctx, w, state, lam_next, lam, accumulate); break;
        case LBM_PR: launch_adj_t<kPR, PREC>(ctx, w, state, lam_next, lam, accumulate); break;
        case LBM_RR: launch_adj_t<kRR, PREC>(ctx, w, state, lam_next, lam, accumulate); break;
        default: launch_adj_t<kStreamOnly, PREC>(ctx, w, state, lam_next, lam, accumulate); break;
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
    for (int k = 0; k < count; ++k) {
        const int acc = ctx->wslots_live ? 1 : 0;
        switch (ctx->prec) {
            case LBM_F64: launch_adj_p<kF64>(ctx, model, omega, states[k], lam[k], lam[k + 1], acc); break;
            case LBM_F32_SHIFTED: launch_adj_p<kF32>(ctx, model, omega, states[k], lam[k], lam[k + 1], acc); break;
            default: launch_adj_p<kF16>(ctx, model, omega, states[k], lam[k], lam[k + 1], acc); break;
        }
        ctx->wslots_live = true;
    }
    rc = check_hip(hipGetLastError(), "adjoint kernel launch");
    if (rc != LBM_OK || !domega) return rc;
    return lbm_adjoint_flush(ctx, domega);
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
