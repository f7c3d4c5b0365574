/*
 * lbm_adjoint.h - discrete adjoint of the stream-and-collide scheme, and raw state
 * checkpoints for reverse sweeps.
 *
 * Forward map of one step (eq. StreamCollide): f_{n+1} = S C(f_n; omega), C the per-cell
 * collision of Appendix B, S the streaming permutation.  Its adjoint, for a loss L of the
 * final state, is
 *     lambda_n(x) = J_C(f_n(x))^T mu(x),   mu_i(x) = lambda_{n+1, i}(x + xi_i)      (S^T)
 *     dL/domega  += sum_x (dC/domega (f_n(x)))^T mu(x)
 * with J_C = dC/df, the Jacobian whose role in the linear analysis of the paper is set out
 * in Appendix A (eq. Perturbed_Collision).  Here it is applied in transposed form by a
 * hand-written reverse pass of each model's moment transform -> relax -> back-transform,
 * with no matrix formed.  The initial state f_0 = f^eq_N(rho0, u0) pulls lambda_0 back to
 * dL/du0 (lbm_eq_vjp).
 *
 * Arrays
 *   raw state   the context's own storage of one state (9 planes, storage precision,
 *               pre-streamed), lbm_state_bytes bytes; only meaningful to the same context
 *   lambda      adjoint populations, 9 planes [q][y][x] with the context's plane stride
 *               (lbm_adjoint_bytes bytes): FP64 for LBM_F64 contexts, FP32 otherwise
 * All pointers below are device pointers unless stated; work is enqueued on the context's
 * stream.  Conventions otherwise as in lbm.h.
 */
#ifndef LBM_ADJOINT_H
#define LBM_ADJOINT_H

#include <stddef.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of one raw state of this context (0 if ctx is NULL). */
size_t lbm_state_bytes(lbm_ctx* ctx);

/* Bytes of one adjoint population array of this context (0 if ctx is NULL). */
size_t lbm_adjoint_bytes(lbm_ctx* ctx);

/* Copy the current state, in the context's storage format, to dst (lbm_state_bytes bytes).
 * Asynchronous (device-to-device). */
int lbm_save_state(lbm_ctx* ctx, void* dst);

/* Make a raw state saved by lbm_save_state of this context the current state, with step
 * counter `step` (>= 0); the blow-up record is cleared.  Asynchronous. */
int lbm_load_state(lbm_ctx* ctx, const void* src, long long step);

/* One forward step from raw state src (f_n, saved by lbm_save_state or written by this
 * function) to raw state dst (receives f_{n+1}), without touching the context's current state
 * or step counter: reverse sweeps rebuild the states of a segment straight into their
 * checkpoint slots.  src and dst must differ; `step` = n is the index recorded if src has a
 * node with !(rho > 0) (lbm_status).  Asynchronous. */
int lbm_step_raw(lbm_ctx* ctx, int model, const double* omega, const void* src, void* dst,
                 long long step);

/* count (>= 0) independent raw steps in one call, in order: step k reads src[k] and writes
 * dst[k] (src[k] != dst[k]) with step index step0 + k.  src and dst are host arrays of
 * device pointers; a later step may read what an earlier one wrote (stream order).  Same
 * arithmetic as lbm_step_raw, without one host call per step. */
int lbm_step_raw_many(lbm_ctx* ctx, int model, const double* omega, const void* const* src,
                      void* const* dst, int count, long long step0);

/* count (>= 0) pairs of raw steps in one call, in order, each as one launch of the two-step
 * kernel with a ring of 8 rows (strips as in lbm_set_fusion, of the height of the model's two-step
 * tail shape where the context has one (lbm_set_fusion_depth), else of its lbm_set_fusion strip
 * height, 16 rows if fused launches are off): pair k reads src[k] (state step0 + 2k) and writes
 * dst[k] (state step0 + 2k + 2);
 * when mid is non-NULL and mid[k] is non-NULL, the state step0 + 2k + 1 is also written to
 * mid[k].  The states written are bit-identical to those of two lbm_step_raw calls.  src, mid
 * and dst are host arrays of device pointers; the three buffers of a pair must differ. */
int lbm_step2_raw_many(lbm_ctx* ctx, int model, const double* omega, const void* const* src,
                       void* const* mid, void* const* dst, int count, long long step0);

/* count (>= 0) triples of raw steps in one call, in order, each as one launch of the three-step
 * kernel on the model's three-step shape: triple k reads src[k] (state step0 + 3k) and writes dst[k]
 * (state step0 + 3k + 3); the two states between are not written.  The states written are
 * bit-identical to those of three lbm_step_raw calls.  src and dst are host arrays of device
 * pointers, src[k] != dst[k].  LBM_EUNSUPPORTED unless the context runs the model three steps per
 * launch (lbm_set_fusion_depth 3 with a ring of 4 or 8 rows, the default on large FP32 and FP64
 * grids). */
int lbm_step3_raw_many(lbm_ctx* ctx, int model, const double* omega, const void* const* src,
                       void* const* dst, int count, long long step0);

/* Seed of the velocity loss L = || u(f) - u_target ||_2 (sum over nodes and both
 * components) for the current state f:
 *   ux_t, uy_t  device, nx*ny FP64 [y][x]: the target velocity
 *   lam         device, lbm_adjoint_bytes: receives dL/df (u = sum xi f / sum f)
 *   loss        host, 1 double: receives L (computed in FP64)
 * Synchronises the stream (L is needed to scale the seed).  L = 0 gives LBM_EINVAL. */
int lbm_adjoint_seed_velocity_l2(lbm_ctx* ctx, const double* ux_t, const double* uy_t, void* lam,
                                 double* loss);

/* One reverse step through the collision of state f_n and the streaming that follows it:
 *   model, omega  as in lbm_step (must be those of the forward step)
 *   state         raw state f_n (lbm_save_state of this context), or NULL = current state
 *   lam_next      lambda_{n+1} (read); lam: receives lambda_n (must not alias lam_next)
 *   domega        device, LBM_NOMEGA doubles: dL/domega of this step (and of any steps
 *                 left pending by lbm_adjoint_many) is ADDED (FP64, deterministic order)
 * Asynchronous. */
int lbm_adjoint_step(lbm_ctx* ctx, int model, const double* omega, const void* state,
                     const void* lam_next, void* lam, double* domega);

/* count (>= 0) reverse steps in one call: step k applies the adjoint at raw state states[k]
 * to lam[k] and writes lam[k + 1] (host arrays of device pointers; lam has count + 1 entries,
 * lam[k] != lam[k + 1]).  Same arithmetic as lbm_adjoint_step, without one host call per step.
 * With two reverse steps per launch (lbm_set_adjoint_depth), steps k and k + 1 run as one
 * launch wherever lam[k + 2] != lam[k] (taking steps in pairs from k = 0): lambda at step k + 1
 * then stays on chip and lam[k + 1] is NOT written; the values written to lam[k + 2] (and to
 * every lam that is written) are bit-identical to one step per launch.  A caller that cycles
 * through three buffers (lam[k] = buffer k mod 3) gets pairs; two alternating buffers give one
 * step per launch.
 * Rate gradients: each strip of the grid (64 columns by a fixed number of rows per context)
 * keeps a running FP64 sum of its contributions, in step order, across calls, whether steps run
 * one or two per launch.  With domega != NULL the pending sums are added to domega (device,
 * 5 doubles) at the end of the call and cleared; with domega == NULL they stay pending, so
 * that a whole reverse sweep issued in any grouping of calls sums in the same order
 * (bit-identical gradients).  lbm_adjoint_step is this function with count = 1. */
int lbm_adjoint_many(lbm_ctx* ctx, int model, const double* omega, const void* const* states,
                     int count, void* const* lam, double* domega);

/* Reverse steps per launch of lbm_adjoint_many: 1 (the default) or 2 (pairs of reverse steps
 * as one pass that keeps the intermediate adjoint in LDS: 18 s + 18 a bytes per node and pair
 * against 2 (9 s + 18 a), s and a the stored and adjoint value sizes).  Other values give
 * LBM_EINVAL.  lbm_get_adjoint_depth writes the setting to *steps. */
int lbm_set_adjoint_depth(lbm_ctx* ctx, int steps);
int lbm_get_adjoint_depth(lbm_ctx* ctx, int* steps);

/* Add the pending rate-gradient sums (see lbm_adjoint_many) to domega (device, 5 doubles) and
 * clear them; nothing to add leaves domega unchanged.  Asynchronous. */
int lbm_adjoint_flush(lbm_ctx* ctx, double* domega);

/* Pull-back through the initial equilibrium f_0 = f^eq_N(rho0, u0) of the context's order:
 *   rho0, ux0, uy0   device FP64 [y][x]: the initial fields given to lbm_init
 *   lam0             lambda_0 (lbm_adjoint_bytes)
 *   dux, duy         device FP64 [y][x]: receive dL/du0 (overwritten)
 * Asynchronous. */
int lbm_eq_vjp(lbm_ctx* ctx, const double* rho0, const double* ux0, const double* uy0,
               const void* lam0, double* dux, double* duy);

#ifdef __cplusplus
}
#endif

#endif /* LBM_ADJOINT_H */
