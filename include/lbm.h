/*
 * lbm.h - C ABI of the MI355X (gfx950) D2Q9 stream-and-collide library (liblbm.so).
 *
 * The method is the periodic stream-and-collide lattice Boltzmann scheme
 *     f_i(x + xi_i, t + 1) = f*_i(x, t)                                (eq. StreamCollide)
 * with the post-collision populations f* produced by one of the collision models of
 * Coreixas, Wissocq, Chopard & Latt (2020), Appendix B: each is a per-cell moment transform,
 * a relaxation toward the (extended) equilibrium, and a back-transform to populations.
 *
 * Conventions shared by every entry point
 *   - Lattice: D2Q9, velocities in the index order
 *       i = 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1),
 *     c_s^2 = 1/3 (Section 2 and eq. extendedFeq).
 *   - Grid: nx x ny nodes, periodic in both directions.  Scalar fields are [y][x] row-major
 *     (x fastest), FP64.  Population arrays exchanged with the caller are [q][y][x], FP64.
 *   - State: the state at step n is the PRE-collision populations f(., n).  One step is
 *     collide-then-stream.  The initial state is f(., 0) = f^eq_N(rho(x), u(x)).
 *   - Pointers documented "device" must be device memory of the current HIP device (for
 *     example torch CUDA tensors); "host" pointers are ordinary CPU memory.
 *   - Every function returns LBM_OK (0) or a negative status and never throws or aborts;
 *     lbm_last_error() gives a message for the last failure on the calling thread.
 *   - Asynchrony: work is enqueued on the stream given at lbm_init (NULL = default stream).
 *     Functions that return host values (lbm_moments, lbm_status) synchronise that stream.
 *   - Threading: one context must not be used by two threads at the same time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_Q 9
#define LBM_NOMEGA 5 /* {omega_nu, omega_b, omega_21, omega_12, omega_22} */

/* Collision models (Appendix B).  LBM_STREAM_ONLY copies f* = f (exact permutation test). */
enum {
    LBM_BGK = 0, /* single relaxation toward f^eq_N with omega_nu                          */
    LBM_RM = 1,  /* raw moments, eq. RMcoll                                                 */
    LBM_HM = 2,  /* Hermite moments, relaxed then mapped by eq. HM2RM_Q9                    */
    LBM_CM = 3,  /* central moments (equilibrium order 4 only)                              */
    LBM_CHM = 4, /* central Hermite moments, eq. CHMcoll / eq. CHM2HM_Q9 (order 4 only)     */
    LBM_K = 5,   /* cumulants (order 4 only)                                                */
    LBM_PR = 6,  /* standard regularisation = HM with omega_21 = omega_12 = omega_22 = 1     */
    LBM_RR = 7,  /* recursive regularisation, eq. HMColl_Q9 with eq. RRformulas_D2Q9        */
    LBM_STREAM_ONLY = 99
};

/* Storage precision of the populations. */
enum {
    LBM_F64 = 0,         /* f_i stored in FP64, FP64 arithmetic                               */
    LBM_F32_SHIFTED = 1, /* h_i = f_i - w_i rho0 stored in FP32 (or - f^eq(rho0, U), see
                            lbm_init_shifted), FP32 arithmetic, FP64 rho                         */
    LBM_F16_SHIFTED = 2  /* h_i stored in FP16, FP32 arithmetic (FP32 mass sum)              */
};

/* Status codes. */
enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* bad argument (size, pointer, rate, model/precision code)          */
    LBM_EUNSUPPORTED = -2,/* valid but unsupported combination (e.g. CM with eq_order < 4)     */
    LBM_EHIP = -3,        /* a HIP runtime call or kernel launch failed                        */
    LBM_ESTATE = -4       /* context not initialised / wrong state                             */
};

typedef struct lbm_ctx lbm_ctx; /* opaque, host-side, owned by the library */

/* Bytes of device memory the caller must provide for the populations of an nx x ny grid at
 * precision prec (two copies of the nine population planes, each plane rounded up to 256 bytes
 * plus a 1 KiB skew).
 * Returns 0 for invalid arguments. */
size_t lbm_population_bytes(int nx, int ny, int prec);

/* Create a context and set f(., 0) = f^eq_N(rho, u) (eq. extendedFeq; N = eq_order, the
 * Hermite equilibrium truncated above order N: 2 = standard second order, 3 = with A21/A12,
 * 4 = extended product form).
 *   out        host: receives the new context (NULL on failure)
 *   nx, ny     grid size, each >= 2, nx * ny * 9 < 2^31
 *   prec       LBM_F64 / LBM_F32_SHIFTED / LBM_F16_SHIFTED
 *   eq_order   2, 3 or 4
 *   rho0       reference density; shifted precisions store f_i - w_i rho0 (must be > 0);
 *              ignored by LBM_F64, which stores f_i unshifted
 *   rho,ux,uy  device, nx*ny FP64 each, [y][x]: initial density and velocity (read only,
 *              not retained)
 *   pop_buf    device, caller-owned, >= lbm_population_bytes(nx, ny, prec) bytes, 256-byte
 *              aligned; must stay allocated until lbm_destroy
 *   pop_bytes  size of pop_buf in bytes
 *   hip_stream hipStream_t on which all work of this context is enqueued (NULL = default)
 * The library allocates only a small reduction scratch; it never frees pop_buf. */
int lbm_init(lbm_ctx** out, int nx, int ny, int prec, int eq_order, double rho0,
             const double* rho, const double* ux, const double* uy, void* pop_buf,
             size_t pop_bytes, void* hip_stream);

/* As lbm_init, with the shifted precisions storing h_i = f_i - f^eq_N(rho0, U)_i for a
 * reference velocity U = (ux0, uy0) (|U| < 1) instead of the rest state: for a flow with a
 * mean velocity, U = that mean keeps the stored deviations, and so the FP32 / FP16 rounding,
 * several times smaller.  rho0 and U are rounded to FP32 once; every kernel and the FP64
 * state exchange use the rounded values.  LBM_F64 ignores rho0 and U (unshifted storage).
 * lbm_init(...) is lbm_init_shifted(..., rho0, 0, 0, ...). */
int lbm_init_shifted(lbm_ctx** out, int nx, int ny, int prec, int eq_order, double rho0,
                     double ux0, double uy0, const double* rho, const double* ux,
                     const double* uy, void* pop_buf, size_t pop_bytes, void* hip_stream);

/* Advance nsteps >= 0 steps of stream-and-collide with the given model (eq. StreamCollide).
 *   omega  host, LBM_NOMEGA doubles in [0, 2]: (omega_nu, omega_b, omega_21, omega_12,
 *          omega_22).  omega_nu = 1 / (nu / c_s^2 + 1/2) (Section 4c).  The paper's SRT
 *          preset is all five equal to omega_nu; its REG preset is omega_b = omega_nu and
 *          omega_21 = omega_12 = omega_22 = 1.  BGK uses omega_nu only; PR ignores the last
 *          three (forced to 1).
 * CM, CHM and K require eq_order == 4 (LBM_EUNSUPPORTED otherwise).
 * Every step also checks the state it reads for a node with !(rho > 0) (this catches NaN);
 * the first such step is reported by lbm_status.  Asynchronous. */
int lbm_step(lbm_ctx* ctx, int model, const double* omega, int nsteps);

/* Macroscopic fields of the current state f(., n) and their totals.
 *   rho, ux, uy  device, nx*ny FP64 each, [y][x], or NULL to skip a field
 *   totals       host, 6 doubles or NULL: {sum rho, sum rho ux, sum rho uy,
 *                sum rho |u|^2 / 2, mean |u|^2 (unweighted domain mean), n}
 * rho = sum_i f_i and rho u = sum_i xi_i f_i (eq. RMcoll), all in FP64.  Synchronises the
 * stream when totals != NULL. */
int lbm_moments(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* totals);

/* For callers that cannot allocate device memory or synchronise (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lbm_moments with the six totals written
 * to device memory, asynchronously, and its reduction partials kept in a static device array of
 * the library instead of the context's own scratch.  No allocation and no synchronisation.
 *   ctx          a context made by lbm_init / lbm_init_shifted (outside the no-allocation region)
 *   rho, ux, uy  device, nx*ny FP64 each, [y][x], or NULL: as lbm_moments
 *   totals       device, 6 doubles, or NULL: the same six values lbm_moments returns on the
 *                host, summed in the same order (identical results)
 * Limit: grids whose per-cell launch has at most 65536 blocks of 256 nodes (16.7 M nodes, e.g.
 * 4096 x 4096); larger grids get LBM_EINVAL.  The static array (2.5 MiB per device, held until
 * the process ends) is shared by every context on a device and keeps the last call's partial
 * sums; calls on one device that overlap in time (other streams or threads) race.  Calls in
 * order on one stream are safe. */
int lbm_moments_noalloc(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* totals);

/* Step counter n of the current state and the first step whose state had a node with
 * !(rho > 0) (-1 if none so far).  A bad state n is detected when it is next read: by
 * lbm_step (state n is read by the step that leaves it) or by lbm_moments.
 * Synchronises the stream.  step and blowup_step are host pointers, either may be NULL. */
int lbm_status(lbm_ctx* ctx, long long* step, long long* blowup_step);

/* Copy the current state f(., n) out as unshifted FP64 populations.
 *   f  device, 9*nx*ny FP64, [q][y][x].  Asynchronous. */
int lbm_get_state(lbm_ctx* ctx, double* f);

/* Replace the current state by f (device, 9*nx*ny FP64, [q][y][x], unshifted) and set the
 * step counter to step (>= 0).  The blow-up record is cleared.  Asynchronous. */
int lbm_set_state(lbm_ctx* ctx, const double* f, long long step);

/* Launch shape of the step kernel for one model (model code, or LBM_STREAM_ONLY):
 *   rows  nodes per thread along y: 1, 2 or 4
 *   xcd   0 = hardware block order, 1 = blocks renumbered so that each of the eight XCDs
 *         owns one contiguous band of tiles
 * Results do not depend on the shape (every node is computed by the same arithmetic). */
int lbm_set_launch(lbm_ctx* ctx, int model, int rows, int xcd);

/* Two steps per pass over memory (temporal blocking) for one model (model code, or
 * LBM_STREAM_ONLY): lbm_step then advances two steps per launch, reading and writing each
 * population once per pair of steps instead of twice; an odd last step uses the single-step
 * kernel.  A workgroup owns a strip of columns (128 for an FP32 context when that still gives at
 * least 1024 strips, 64 otherwise) and strip_rows rows and walks down it ring_rows rows at a time,
 * keeping the first step's values of ring_rows + 2 rows (and one halo column each side) in LDS;
 * the halo nodes are collided by both strips that need them.
 *   ring_rows   0 (off), 4, 8 or 16
 *   strip_rows  positive multiple of ring_rows (ignored when ring_rows is 0)
 * A new context starts with ring_rows 8 and strip_rows
 *   FP32: 16 if that gives at least 256 strips, else off;
 *   FP64: 64 if that gives at least 1024 strips, else as FP32;
 *   FP16: 40 if that gives at least 1024 strips, else off;
 * except where an FP32 model's measured best setting on 128-column strips, (ring_rows, strip_rows)
 * = (8, 8) for BGK and (4, 20) for the others, gives at least 1024 such strips: it starts with that;
 * and an FP32 or FP64 context starts every model with three steps per launch
 * (lbm_set_fusion_depth) when its 64-column strips of h rows number at least 512, h being
 * ceil(nx / 64) ny / sqrt(nx ny) rounded to a multiple of 8 and clamped to [8, 64] (n / 64 on an
 * n x n grid), and 128 instead of 64 in FP32: FP32 with ring_rows 8 and strip_rows h, raised in
 * steps of 8 while the strips number more than one round of workgroups (3 per CU) but no more than
 * 1.5 rounds; FP64 with ring_rows 8 and strip_rows h (128 instead of 64).
 * Results are bit-identical to single steps (same arithmetic per node; the LDS ring holds the
 * stored type).  Returns LBM_EINVAL for other values. */
int lbm_set_fusion(lbm_ctx* ctx, int model, int ring_rows, int strip_rows);

/* The two-step setting of `model` (host pointers, either may be NULL; ring_rows 0 = off). */
int lbm_get_fusion(lbm_ctx* ctx, int model, int* ring_rows, int* strip_rows);

/* Steps per fused launch of `model`: 2 (the default) or 3.  With 3, and ring_rows 4 or 8 set by
 * lbm_set_fusion, lbm_step advances three steps per launch (then pairs, then single steps), each
 * the step of eq. StreamCollide: a second LDS ring holds the second step's values, so each
 * population is read and written once per three steps; the first step covers two halo rows and
 * columns on each side of the strip, the second one.  Strips are 64 columns wide in FP32 and 48 in
 * FP64 (the strip and its halo columns fit one wave); with ring_rows 8 a workgroup runs 8 waves, one
 * row each per pass.  Two steps left over by the three-step launches of a new context's default
 * setting run as one two-step launch on a shape of their own: ring_rows 8 on strips (as in
 * lbm_set_fusion) of the smaller of the two-step default height and strip_rows rows; lbm_set_fusion drops that shape
 * (its own shape then takes them), and lbm_autotune keeps its fastest two-step shape for them when
 * that beats single steps.  Bit-identical to single steps.  LBM_EUNSUPPORTED for 3 on an FP16
 * context or on a grid narrower or lower than 2; LBM_EINVAL for other values. */
int lbm_set_fusion_depth(lbm_ctx* ctx, int model, int steps);

/* Steps per fused launch of `model` (host pointer, may be NULL). */
int lbm_get_fusion_depth(lbm_ctx* ctx, int model, int* steps);

/* Autotune the launches of `model` on this context's grid: every single-step shape
 * (rows in {1, 2, 4} x xcd in {0, 1}), the two-step shapes (ring_rows, strip_rows) in
 * {(8, 8), (8, 16), (8, 40), (8, 64), (16, 16), (4, 16), (4, 20), (4, 64)} and, except for FP16,
 * the three-step shapes {(4, 8), (4, 16), (4, 32), (4, 64), (8, 8), (8, 16), (8, 24), (8, 32),
 * (8, 64), (8, 80), (8, 96), (8, 128)} are timed with HIP
 * events over `trials` (>= 1) launches that recompute from the same input copy, so the state, the
 * step counter and the blow-up record are unchanged.  The fastest single-step shape is kept (it
 * also takes the last steps that do not fill a fused launch) and returned through rows_out /
 * xcd_out; the fastest fused shape per step is kept (lbm_get_fusion, lbm_get_fusion_depth) when it
 * beats it, and fusion is switched off otherwise.  us_per_step is the best time per step.  Host
 * pointers, each may be NULL.  Synchronises. */
int lbm_autotune(lbm_ctx* ctx, int model, const double* omega, int trials, int* rows_out,
                 int* xcd_out, double* us_per_step);

/* Release the context (not pop_buf).  NULL is accepted.  Synchronises the stream. */
void lbm_destroy(lbm_ctx* ctx);

/* Message for the last failure on the calling thread ("" if none).  Owned by the library,
 * valid until the next call on this thread. */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
