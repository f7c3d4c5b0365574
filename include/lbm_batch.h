/*
 * lbm_batch.h - many independent periodic D2Q9 simulations advanced by one persistent launch.
 *
 * Each instance is a stream-and-collide run (eq. StreamCollide) with its own grid size,
 * collision model (Appendix B), equilibrium order and relaxation rates, as in the paper's
 * numerical stability study (Section 5b-c: one simulation per (model, Ma, nu) point, with a
 * blow-up test).  Instances share nothing; their nodes are cut into tiles of 256 consecutive
 * nodes, and one persistent grid of co-resident workgroups sweeps all tiles of all instances
 * every step, with a barrier between steps.  The grid is launched cooperatively and sized from the
 * persistent kernel's own resources (VGPRs, LDS, threads against what one CU holds; see
 * lbm_batch_residency), so that all its workgroups are resident together.  As a safety net, the
 * first run of each launch shape probes that size with non-advancing steps under a short barrier
 * bound and lowers it if the grid did not pass every barrier; every barrier wait of the kernel is
 * bounded in wall-clock time, so a grid that is not resident can fail a run with an error but not
 * hang it.
 *
 * Per-instance arithmetic is exactly that of lbm_step (same device code, same rounding): an
 * instance of the batch is bit-identical to the same run through lbm_init / lbm_step.
 * Blow-up: at every step each instance's state is checked for a node with !(rho > 0); the
 * first such step is recorded and the instance is frozen from the next step on.
 *
 * Conventions (grid layout, state, pointers, errors, streams) are those of lbm.h.
 */
#ifndef LBM_BATCH_H
#define LBM_BATCH_H

#include <stddef.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One instance. */
typedef struct {
    int nx, ny;                /* grid, each >= 2 */
    int model;                 /* LBM_BGK .. LBM_RR (not LBM_STREAM_ONLY) */
    int eq_order;              /* 2, 3 or 4 (4 for CM, CHM, K) */
    double omega[LBM_NOMEGA];  /* (omega_nu, omega_b, omega_21, omega_12, omega_22) in [0, 2] */
    double rho0;               /* shifted precisions store f - f^eq_N(rho0, U) (rho0 > 0)    */
    double ux0, uy0;           /* reference velocity U (|U| < 1; 0 = rest), see               */
                               /* lbm_init_shifted; both ignored in FP64                      */
} lbm_instance_desc;

typedef struct lbm_batch lbm_batch; /* opaque, host-side, owned by the library */

/* Bytes of device memory for the populations of all n instances at precision prec (two
 * copies, every instance's planes rounded up to 256 bytes plus a 1 KiB skew).  0 for invalid
 * arguments. */
size_t lbm_batch_population_bytes(const lbm_instance_desc* desc, int n, int prec);

/* Create a batch and set every instance to f^eq(rho, u) of its own equilibrium order.
 *   desc        host, n descriptors (copied)
 *   prec        LBM_F64 / LBM_F32_SHIFTED / LBM_F16_SHIFTED
 *   rho,ux,uy   device FP64: the initial fields of all instances concatenated in instance
 *               order, each instance's block [y][x] (sum of nx*ny values each); read only
 *   pop_buf     device, caller-owned, >= lbm_batch_population_bytes bytes, 256-byte aligned
 *   hip_stream  stream for all work of this batch (NULL = default)
 * Allocates descriptor and tile tables, the barrier counter, the blow-up record and the
 * per-instance flags (O(number of tiles) bytes).  LBM_EUNSUPPORTED if the device has no
 * cooperative launches. */
int lbm_batch_create(lbm_batch** out, const lbm_instance_desc* desc, int n, int prec,
                     const double* rho, const double* ux, const double* uy, void* pop_buf,
                     size_t pop_bytes, void* hip_stream);

/* Advance every live instance by nsteps >= 0 steps in one cooperative persistent launch (with
 * two steps per pass on, lbm_batch_set_fusion: the first 4 * (nsteps / 4) steps in a launch of
 * the two-step kernel, the rest in one of the single-step kernel; with three steps per pass,
 * lbm_batch_set_fusion_depth: the first 3 * (nsteps / 3) steps in a launch of the three-step
 * kernel, the rest one step per pass).
 * Asynchronous, except that the first run of each launch shape first probes how many workgroups
 * per CU really stay co-resident (the runtime's occupancy figure can be one too high): two
 * non-advancing steps with a 250 ms barrier bound per candidate, from the occupancy figure
 * down; this synchronises the stream and leaves states and records unchanged.  A refused launch
 * returns LBM_EHIP.  A grid barrier that does not complete within two seconds stops the launch
 * (every wave exits); lbm_batch_status then reports LBM_EHIP. */
int lbm_batch_run(lbm_batch* b, int nsteps);

/* Step counter and, per instance, the first step whose state had a node with !(rho > 0)
 * (-1 if none).  blowup_steps: host, n values, or NULL.  Synchronises the stream. */
int lbm_batch_status(lbm_batch* b, long long* step, long long* blowup_steps);

/* Current state of one instance as unshifted FP64 populations (device, 9*nx*ny, [q][y][x]).
 * An instance that blew up at step b stops at the state its last pass wrote: state b + 1 (the
 * collided state of step b) when that pass took one step, the end of the pair containing b
 * (b + 1 or b + 2) when it took two; either way not a meaningful flow state.  One retired at step
 * r (lbm_batch_set_active) stops at state r.  Synchronises the stream (to read those records),
 * then enqueues the copy. */
int lbm_batch_get_state(lbm_batch* b, int instance, double* f);

/* Domain mean of |u|^2 of every instance's current state, the quantity of the stability
 * criterion of Section 5b (unweighted mean over the nx*ny nodes, u = j / rho in FP64):
 *   mean_u2   device, n doubles (overwritten), in instance order
 * Deterministic (fixed summation order).  Values of blown-up or retired instances are
 * unspecified (NaN for blown-up states).  Asynchronous. */
int lbm_batch_mean_u2(lbm_batch* b, double* mean_u2);

/* Retire instances: active is a device array of n ints; every instance whose flag is 0 is
 * retired for good from the following lbm_batch_run calls (its state and blow-up record stay as
 * they are, and the current step is recorded as its last).  Nonzero flags change nothing: a
 * retired instance cannot be re-admitted.  All instances start active.  The flags are read in
 * stream order (the array may be overwritten once the stream has passed this call).
 * Asynchronous. */
int lbm_batch_set_active(lbm_batch* b, const int* active);

/* Re-deal the live instances (neither blown up nor retired) over the XCDs, largest first, so that
 * every XCD keeps a similar number of nodes to advance as instances drop out; instances that are
 * no longer live leave the per-XCD work lists.  Results are unchanged: an instance's arithmetic is
 * the same on every XCD.  Synchronises the stream. */
int lbm_batch_rebalance(lbm_batch* b);

/* Launch shape of the persistent kernel: nodes per thread per tile (1, 2 or 4) and resident
 * workgroups per CU (1 .. the probed residency limit; 0 = that limit).  Takes effect at the next
 * lbm_batch_run. */
int lbm_batch_set_launch(lbm_batch* b, int nodes_per_thread, int groups_per_cu);

/* Two steps per pass of the persistent kernel (temporal blocking, as lbm_set_fusion for a single
 * grid): strip_rows 0 = off (the default), else a positive multiple of 8: each instance is cut
 * into strips of 64 columns and strip_rows rows, one workgroup advances a strip two steps with
 * the first step's values in an LDS ring (halo nodes are collided by both strips that need
 * them), and the workgroups of an XCD meet at one barrier per pair of steps.  Runs of 4 steps
 * use it (see lbm_batch_run).  Every live instance stays bit-identical to its single-step (and
 * plain) run and its blow-up step is the same; the state left by a blown-up instance may differ
 * (see lbm_batch_get_state).  Synchronises the stream when strip_rows changes. */
int lbm_batch_set_fusion(lbm_batch* b, int strip_rows);

/* The current strip height of two steps per pass (0 = off); strip_rows is a host pointer. */
int lbm_batch_get_fusion(lbm_batch* b, int* strip_rows);

/* Steps per fused pass (with lbm_batch_set_fusion on): 2 (the default) or 3.  With 3 a workgroup
 * advances a strip three steps (eq. StreamCollide each) with the first and second steps' values in
 * two LDS rings of 6 rows (as lbm_set_fusion_depth for a single grid), and the workgroups of an XCD
 * meet at one barrier per three steps; any number of triples keeps the states in the copy of their
 * step's parity.  FP64 strips are 48 columns wide (strip and halo fit one wave), FP32 strips 64.
 * Bit-identical to single steps, blow-up steps included.  LBM_EUNSUPPORTED for 3 on
 * an FP16 batch; LBM_EINVAL for other values. */
int lbm_batch_set_fusion_depth(lbm_batch* b, int steps);

/* Steps per fused pass (host pointer, may be NULL). */
int lbm_batch_get_fusion_depth(lbm_batch* b, int* steps);

/* Residency of launch shape `shape` (0, 1, 2: one step per pass with 1, 2, 4 nodes per thread;
 * 3: two steps per pass; 4: three steps per pass): the workgroups per CU that the persistent
 * kernel's resources allow, the runtime's occupancy figure, the figure confirmed by the first run
 * of that shape (0 before it), and how many residency probes of this batch had to lower a figure.
 * Host pointers, each may be NULL.  Does not synchronise. */
int lbm_batch_residency(lbm_batch* b, int shape, int* from_resources, int* occupancy_query, int* resident,
                        int* probe_stepdowns);

/* Autotune the persistent launch: each candidate (nodes per thread in {1, 2, 4}, or two or, for
 * FP64 and FP32, three steps per pass at the current strip height (64 rows unless set), x groups
 * per CU in {limit, limit/2}, limit = the probed residency limit of that shape) runs `trials`
 * (>= 1) steps, pairs or triples that all recompute from the same input copy, so states and
 * counters are unchanged, and the blow-up records are restored afterwards.  Keeps the fastest per
 * step: it sets nodes per thread, groups per CU and whether two or three steps per pass are used
 * (lbm_batch_get_fusion, lbm_batch_get_fusion_depth), and returns the first two and the time per
 * step.  Synchronises. */
int lbm_batch_autotune(lbm_batch* b, int trials, int* nodes_per_thread, int* groups_per_cu,
                       double* us_per_step);

/* Release the batch (not pop_buf).  NULL is accepted.  Synchronises the stream. */
void lbm_batch_destroy(lbm_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_BATCH_H */
