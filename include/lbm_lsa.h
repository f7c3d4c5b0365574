/*
 * lbm_lsa.h - linear stability analysis of the stream-and-collide scheme (Section 4, Appendix A).
 *
 * About a uniform flow f = f^eq_N(rho = 1, U), a perturbation f' obeys (eq. DiscretePerturbedEq)
 *     f'_i(x + xi_i, t + 1) = [delta_ij + J_ij] f'_j(x, t),
 * where delta + J is the Jacobian of the post-collision populations with respect to the
 * pre-collision ones (eq. Perturbed_Collision), here called J_C.  A plane wave f' = A exp(i(k.x -
 * omega t)) turns this into the eigenvalue problem (eq. EigenvaluePbDiscrete)
 *     M(k) A = exp(-i omega) A,   M(k) = E(k) J_C,   E(k) = diag(exp(-i xi_i . k)),
 * so a wave grows at the rate Im(omega) = log |lambda| and the scheme is linearly stable for a
 * given flow when every eigenvalue lambda of every M(k) has |lambda| <= 1.
 *
 * J_C is obtained from the library's own collision code (its hand-written reverse mode, one
 * unit vector per row) in FP64; the eigenvalues come from a complex Hessenberg reduction and
 * shifted QR iteration, one wave number per thread.
 *
 * Points: the lattice order of the populations and the rate vector are those of lbm.h.  All
 * array arguments are device pointers; calls synchronise the stream (they copy the points in
 * and release their scratch) unless stated.  Errors as in lbm.h.
 */
#ifndef LBM_LSA_H
#define LBM_LSA_H

#include <stddef.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One base flow and collision operator. */
typedef struct {
    int model;                 /* LBM_BGK .. LBM_RR */
    int eq_order;              /* 2, 3 or 4 (4 for CM, CHM, K) */
    double omega[LBM_NOMEGA];  /* (omega_nu, omega_b, omega_21, omega_12, omega_22) in [0, 2] */
    double ux, uy;             /* mean flow U (|U| < 1), density 1 */
} lbm_lsa_point;

/* J_C of each of the npts points (host array):
 *   J   device, npts * 81 doubles, point-major, row-major: J[p][i][j] = d f*_i / d f_j at
 *       f = f^eq_N(1, U) */
int lbm_lsa_jacobian(const lbm_lsa_point* pts, int npts, double* J, void* hip_stream);

/* The nine eigenvalues of M(k) for one point and nk wave numbers:
 *   kx, ky   device, nk doubles each (radians per node)
 *   lam      device, nk * 9 * 2 doubles: (re, im) of the eigenvalues of M(k[q]) at
 *            lam[(q * 9 + m) * 2], unordered.  An eigenvalue iteration that does not converge
 *            gives NaN for that wave number. */
int lbm_lsa_eigenvalues(const lbm_lsa_point* pt, const double* kx, const double* ky, int nk,
                        double* lam, void* hip_stream);

/* Spectral radius max_m |lambda_m(M(k))| for every (point, wave number) pair:
 *   pts      host, npts points;  kx, ky  device, nk doubles each
 *   radius   device, npts * nk doubles, point-major (NaN where the iteration did not converge) */
int lbm_lsa_radius(const lbm_lsa_point* pts, int npts, const double* kx, const double* ky, int nk,
                   double* radius, void* hip_stream);

/* Linear stability of the discrete-velocity Boltzmann equation with BGK collisions (Section 3c,
 * Appendix A, eq. EigenvaluePbContinuous): about the same base flows, a plane wave
 * A exp(i (k . x - omega t)) obeys M^C(k) A = omega A with
 *     M^C(k) = diag(xi_i . k) + i J^C,   J^C = -(I - F) / tau,   F = d f^eq_N / d f at f^eq_N(1, U),
 * (F is taken from the library's BGK collision at omega = 1, whose post-collision state is f^eq),
 * and the wave grows when Im(omega) > 0.
 *   pts      host, npts points (only eq_order, ux, uy are used)
 *   tau      relaxation time > 0 (the growth rates scale with it; stability does not depend on it)
 *   kx, ky   device, nk doubles each
 *   growth   device, npts * nk doubles, point-major: max_m Im(omega_m(k)) (NaN where the
 *            eigenvalue iteration did not converge) */
int lbm_lsa_dvbe_growth(const lbm_lsa_point* pts, int npts, double tau, const double* kx, const double* ky,
                        int nk, double* growth, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_LSA_H */
