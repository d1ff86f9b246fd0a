/*
 * cn_aao2d.h -- C ABI of the all-at-once Crank-Nicolson system and the
 * alpha-circulant preconditioner for a 2D spatial operator.
 *
 * The 2D experiments of Sec. 5 (the Heston operator, eq. (5.1), and the
 * SABR operator) discretise a spatial operator on an N_x x N_y tensor grid;
 * the all-at-once matrix (eq. (2.2)) and the preconditioner (eq. (3.1)) are
 * built from A~ = tau A exactly as in one dimension, and step (b) of
 * eq. (3.2) becomes one complex-shifted sparse solve
 * (lambda_{1,j} I - lambda_{2,j} A~) per frequency j.
 *
 * The operator: nine coefficient arrays of N_x N_y doubles (device),
 * stencil[q * N_x N_y + i], q = 3 (dy + 1) + (dx + 1), dy, dx in {-1, 0, 1}:
 * row i of A (grid point (iy, ix), i = iy N_x + ix, x fastest) has
 * stencil[q, i] in the column of grid point (iy + dy, ix + dx); entries
 * whose neighbour lies outside the grid are ignored (homogeneous Dirichlet
 * data outside).  This covers central differences of second-order operators
 * with a mixed derivative (the form of eq. (5.1)).
 *
 * Vectors: a space-time vector holds N_t blocks of N_x N_y doubles, element
 * (k, i) at k N_x N_y + i (level t_{k+1}), device memory owned by the caller.
 *
 * Step (b): each shifted matrix mu_j I - A~ (mu_j = lambda_{1,j} /
 * lambda_{2,j}, j = 0..N_t/2; the other half by conjugate symmetry,
 * Remark 1) is factored once at creation by band Gaussian elimination in
 * complex128 without pivoting (half-bandwidth N_x + 1 in the x-fastest
 * ordering) and applied per call by forward and back substitution.  No
 * pivoting is sound when the shifted matrices are diagonally dominant
 * (Re mu_j > 0 and A with a non-positive diagonal dominating its row, the
 * case of central differences at cell Peclet numbers below 2 without a
 * mixed derivative); a pivot below 1e-12 of its row's scale is reported as
 * CN_ESINGULAR at creation.
 *
 * Limits: 1 <= N_x <= 127, N_y >= 1, N_x N_y <= 8192 (the substitution
 * keeps one frequency's vector in LDS), N_t a power of two in [1, 1024].
 * Workspace: (N_t/2 + 1) N_x N_y (2 N_x + 3) complex128 (the band factors)
 * plus (N_t/2 + 1) N_x N_y complex128 (the spectrum), and the same again
 * for the band during set-up.
 *
 * Errors and streams: as cn_aao.h (cn_status codes, cn_last_error()); calls
 * enqueue on the problem's stream without synchronising, except cn2d_create
 * (synchronises after set-up).
 */
#ifndef CN_AAO2D_H
#define CN_AAO2D_H

#include <stdint.h>

#include "cn_aao.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny;          /* grid: N_x in [1, 127], N_y >= 1, N_x N_y <= 8192 */
    int32_t nt;              /* time steps: power of two in [1, 1024]         */
    int32_t m_max;           /* largest GMRES restart length, 0..64 (0: no     */
                             /* solver workspace)                             */
    double T;                /* final time, > 0 (tau = T / N_t)               */
    double alpha;            /* 0 < alpha < 1                                 */
    const double *stencil;   /* device, 9 N_x N_y coefficients of A           */
    void *stream;            /* hipStream_t (NULL: the null stream)           */
} cn2d_problem;

typedef struct cn2d cn2d;

/* Validate p, copy the stencil, build the time tables and factor the
 * N_t/2 + 1 shifted band matrices.  CN_EINVAL for sizes or alpha out of
 * range, CN_ENOMEM when the workspace does not fit, CN_ESINGULAR for a
 * vanishing pivot. */
cn_status cn2d_create(const cn2d_problem *p, cn2d **out);
cn_status cn2d_destroy(cn2d *h);

/* y = M x (eq. (2.2), block form of Sec. 3.2); x != y. */
cn_status cn2d_matvec(cn2d *h, const double *x, double *y);

/* b = xi + tau f (eq. (2.2)): u0 N_x N_y values, f N_t blocks f^{k+1/2}. */
cn_status cn2d_rhs(cn2d *h, const double *u0, const double *f, double *b);

/* z = P_alpha^{-1} v by the three steps of eq. (3.2) in complex128; v == z
 * allowed. */
cn_status cn2d_pc_apply(cn2d *h, const double *v, double *z);

/* GMRES for M u = b (right-preconditioned flexible GMRES(m) with P_alpha,
 * Sec. 5's solver, as cn_gmres_solve): classical Gram-Schmidt applied twice
 * in two passes of dots and updates, the Hessenberg column, Givens rotations
 * and the triangular solve on the device; the host waits once per inner
 * iteration for the residual estimate.  opts->m <= m_max; use_x0 0 (x is
 * zeroed) or 1; flags and err_tol must be 0.  x: initial guess / solution
 * (b = 0 gives x = 0 at once).
 * info (may be NULL): iterations, restarts, products, relres_true from the
 * recomputed residual.  CN_NOT_CONVERGED when max_iters is spent.
 * Workspace (at create, m_max > 0): (2 m_max + 2) N_t N_x N_y doubles. */
cn_status cn2d_gmres_solve(cn2d *h, const double *b, double *x, const cn_gmres_opts *opts,
                           cn_gmres_info *info);

/* Thread-local message of the last failed cn2d_* call on this thread. */
const char *cn2d_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
