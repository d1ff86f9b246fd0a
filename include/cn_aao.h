/*
 * cn_aao.h -- C ABI of the MI355X all-at-once Crank-Nicolson solver with the
 * generalized block-circulant (alpha-circulant) preconditioner.
 *
 * Mathematics (arXiv 2401.16113):
 *   - CN scheme, eq. (2.1): (u^{k+1}-u^k)/tau = A (u^{k+1}+u^k)/2 + f^{k+1/2},
 *     tau = T/N_t, f evaluated at t_{k+1/2}.
 *   - All-at-once system, eq. (2.2): M u = b,  M = B1 (x) I - B2 (x) A~,
 *     A~ = tau A, B1 = tridiag(-1,1,0), B2 = tridiag(1,1,0)/2,
 *     b = xi + tau f, xi = [(I + A~/2) u^0; 0; ...; 0].
 *     Block form (Sec. 3.2): (M u)^1 = Q1 u^1, (M u)^k = Q1 u^k - Q2 u^{k-1},
 *     Q1 = I - A~/2, Q2 = I + A~/2.
 *   - Preconditioner, eq. (3.1): P_alpha = C1^(alpha) (x) I - C2^(alpha) (x) A~,
 *     applied by the three steps of eq. (3.2) (alpha-weighted DFT along time,
 *     N_t shifted spatial solves, inverse DFT), halved by conjugate symmetry
 *     (Remark 1).
 *   - Right-preconditioned restarted GMRES(m), zero initial guess, stop on the
 *     relative residual (Sec. 5).
 *
 * Vector layout (all calls): a space-time vector of n = nx*nt doubles,
 * element (k, i) at k*nx + i, k = 0..nt-1 standing for time level t_{k+1},
 * space fastest (the lexicographic stacking u = [u^1; ...; u^{N_t}] of
 * eq. (2.2)).
 *
 * Memory: every data pointer below is a DEVICE pointer (hipMalloc'ed or a
 * torch tensor's storage) owned by the caller unless stated otherwise.  The
 * handle owns only its own workspace and never frees caller memory.
 *
 * Streams: calls enqueue work on the stream given at creation and return
 * without synchronising, except cn_aao_create (synchronises after set-up),
 * cn_gmres_solve and cn_batch_solve (synchronise before filling `info`).
 *
 * Errors: every entry point returns a cn_status; no C++ exception crosses
 * the ABI.  cn_last_error() returns a thread-local message for the last
 * failure on the calling thread.  A handle is not thread-safe; distinct
 * handles are independent.
 */
#ifndef CN_AAO_H
#define CN_AAO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CN_OK = 0,              /* success                                        */
    CN_NOT_CONVERGED = 1,   /* iteration budget spent; x holds the last iterate */
    CN_EINVAL = -1,         /* invalid argument (sizes, alpha, pointers, ...)  */
    CN_ENOMEM = -2,         /* device workspace does not fit                  */
    CN_EHIP = -3,           /* a HIP runtime call failed                      */
    CN_ESINGULAR = -4       /* a shifted system of step (b) is singular       */
} cn_status;

typedef enum {
    CN_PC_FP64 = 0,         /* preconditioner in float64 / complex128        */
    CN_PC_FP32 = 1          /* preconditioner in float32 / complex64 (flexible GMRES) */
} cn_pc_prec;

/* cn_problem.flags */
#define CN_FLAG_ALLOW_ALPHA_ONE 1  /* accept alpha = 1: the classical block-circulant
                                      preconditioner P_1 (Remark 2); singular
                                      shifted systems then give CN_ESINGULAR   */

typedef struct {
    int32_t nx;             /* spatial unknowns N_x >= 1                       */
    int32_t nt;             /* time steps N_t: power of two in [1, 8192];      */
                            /* N_t * (N_x rounded up to 16) < 2^29            */
    int32_t m_max;          /* largest GMRES restart length used, 1..64        */
    int32_t flags;          /* CN_FLAG_* bits                                  */
    double T;               /* final time, > 0 (tau = T/nt)                    */
    double alpha;           /* alpha of the alpha-circulants, 0 < alpha < 1    */
    const double *a_lo;     /* device, nx: A_{i,i-1} (entry 0 ignored)         */
    const double *a_di;     /* device, nx: A_{i,i}                             */
    const double *a_up;     /* device, nx: A_{i,i+1} (entry nx-1 ignored)      */
    const double *d_half;   /* device, nt, or NULL: time weights d(t_{k+1/2}) of
                               L(t) = d(t) L (Sec. 5.2); the preconditioner then
                               uses their mean times C2^(alpha)                */
    cn_pc_prec pc_prec;     /* precision of the preconditioner                 */
    void *stream;           /* hipStream_t; NULL = the default stream          */
} cn_problem;

typedef struct cn_aao cn_aao;

/* Validate p, copy A~ = tau A and the time weights, build the float64 tables
 * (alpha^{+-k/N_t}, twiddles, lambda_{1,j}/lambda_{2,j} from the
 * diagonalisation of Sec. 3.1), factor the interface systems of the
 * partitioned step-(b) solve and allocate the GMRES workspace for m_max.
 * Returns CN_EINVAL on bad input, CN_ENOMEM if the workspace does not fit,
 * CN_ESINGULAR if a shifted system is singular.  On success *out owns the
 * handle (release with cn_aao_destroy); on failure *out is NULL. */
cn_status cn_aao_create(const cn_problem *p, cn_aao **out);
cn_status cn_aao_destroy(cn_aao *h);

/* b = xi + tau f (eq. (2.2)); u0: nx values; f: nt*nx values f^{k+1/2}
 * (row k = f^{k+1/2}); b: nt*nx.  All device pointers. */
cn_status cn_rhs(cn_aao *h, const double *u0, const double *f, double *b);

/* y = M x (eq. (2.2)).  x and y: n doubles, x != y (CN_EINVAL if they overlap). */
cn_status cn_matvec(cn_aao *h, const double *x, double *y);

/* z = P_alpha^{-1} v by the three steps of eq. (3.2), in the handle's
 * preconditioner precision, float64 input and output.  v == z is allowed. */
cn_status cn_pc_apply(cn_aao *h, const double *v, double *z);

typedef struct {
    int32_t m;              /* restart length, 1 <= m <= m_max                 */
    int32_t max_iters;      /* total inner-iteration budget, >= 1              */
    int32_t use_x0;         /* 0: x0 = 0; 1: x holds the initial guess;        */
                            /* 2: as 1, but an instance whose initial residual */
                            /*    is no smaller than ||b|| starts from x0 = 0  */
    int32_t flags;          /* CN_SOLVE_* bits, 0 for the defaults             */
    double rtol;            /* stop when ||b - M x||_2 / ||b||_2 <= rtol       */
    double err_tol;         /* > 0: error-controlled stopping (below); 0: off  */
} cn_gmres_opts;

/* Error-controlled stopping.  A residual bound does not bound the error: the
 * error of x is M^{-1} r, and for stiff operators max|M^{-1} r| / max|x| can
 * be tens of times ||r|| / ||b||.  With err_tol > 0 (and rtol > 0), each
 * instance first stops at its own target relres <= rt_i <= rtol, where rt_i
 * is remembered by the handle or batch from its previous solve with the same
 * rtol and err_tol (initially min(rtol, err_tol / 10)).  Then every
 * instance's relative max-norm error is estimated as ||r|| max|z| / max|x|
 * with z = P_alpha^{-1} r / ||r|| (one preconditioner apply and one reduction
 * on the final residual; P_alpha^{-1} M = I + O(alpha), so the estimate is within a
 * relative O(alpha) of the error, Sec. 3).  An instance above err_tol
 * continues from its x with rt_i = relres * err_tol / (4 * estimate) (at
 * least halving it) and is estimated again, at most three times; the status
 * is CN_NOT_CONVERGED if an estimate still exceeds err_tol.  The targets
 * only tighten (they start over when rtol or err_tol change).  Counters in
 * cn_gmres_info add up over the continuations; err_est holds the last
 * estimate (-1 when off), err_passes the continuation solves. */

/* cn_batch_solve launches each inner iteration as one captured HIP graph
 * (captured on first use per iteration index, restart length and rtol, and
 * kept with the batch); this flag launches the same kernels one by one. */
#define CN_SOLVE_NO_GRAPHS 1
/* By default cn_batch_solve captures the first K inner iterations of a cycle
 * as one graph, K = the first cycle's iteration count of the batch's last
 * solve (2 <= K <= m), and waits once for the summary of iteration K-1;
 * iterations queued after convergence return at entry, and a cycle that
 * needs more continues one graph per iteration.  This flag keeps one graph
 * per iteration throughout.  Ignored with CN_SOLVE_NO_GRAPHS and by
 * cn_gmres_solve. */
#define CN_SOLVE_ITERATION_GRAPHS 2

typedef struct {
    int32_t iters;          /* inner iterations (= preconditioned matvecs)    */
    int32_t restarts;       /* completed cycles that did not converge         */
    int32_t matvecs;        /* all products with M, residual checks included  */
    int32_t pc_applies;     /* preconditioner applications                    */
    int32_t x0_rejected;    /* 1: use_x0 = 2 replaced the initial guess by 0  */
    int32_t err_passes;     /* continuation solves of error-controlled stopping */
    double relres_true;     /* ||b - M x|| / ||b|| at return (recomputed)      */
    double relres_est;      /* last least-squares residual estimate / ||b||   */
    double seconds;         /* wall time of the call                          */
    double err_est;         /* error estimate (err_tol > 0), else -1          */
} cn_gmres_info;

/* Right-preconditioned restarted GMRES(m) (flexible form: the preconditioned
 * vectors are stored, so x += Z y), Arnoldi by classical Gram-Schmidt with
 * one re-orthogonalisation (CGS2) in float64.  With CN_PC_FP32 the
 * preconditioner runs in float32 and its outputs are stored in float32 and
 * multiplied by M as stored, which keeps the Arnoldi relation M Z = V H.
 * b, x: device, n doubles, b != x.  On return x holds the last iterate and
 * `info` (may be NULL) is filled.  Returns CN_OK when the true relative
 * residual is <= rtol, CN_NOT_CONVERGED when max_iters is spent.  b = 0
 * returns x = 0. */
cn_status cn_gmres_solve(cn_aao *h, const double *b, double *x,
                         const cn_gmres_opts *opts, cn_gmres_info *info);

/* Sizes chosen at creation (for tests and tooling): tile width of the
 * partitioned step-(b) solve, number of tiles, workgroup size of the
 * transform kernels, workgroups per tile of the inverse transform (1 or 2:
 * each inverts half of the tile's columns) and the transforms' split (1, or
 * 2: the forward and the inverse transform each handle the even
 * frequencies, then the odd ones, in half the LDS).  Any pointer may be
 * NULL. */
cn_status cn_aao_query(const cn_aao *h, int32_t *tile_cols, int32_t *tiles,
                       int32_t *threads, int32_t *inverse_split,
                       int32_t *forward_split);

/* Preconditioner apply that allocates nothing, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops or
 * harnesses that forbid hipMalloc).  Computes z = P_alpha^{-1} v as
 * cn_pc_apply does (FP64 input and output, row pitch N_x, v == z allowed)
 * for the problem p, without a handle: p's fields as for cn_aao_create
 * (m_max and flags unused; 0 < alpha < 1), enqueued on p->stream with no
 * synchronisation.  Every table and work array (operator rows, alpha
 * weights, twiddles, shifts, interface factors, tile images, interface and
 * separator values) is built on the device, each call, in a library-owned
 * array of CN_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs
 * on holds until the process ends; a problem that needs more (about 13 bytes
 * per unknown in float32, 25 in float64, plus O(N_t) tables) gets CN_EINVAL.
 * All calls on one GPU share that array and it keeps the last call's
 * contents: calls that overlap on one GPU (concurrent streams, threads)
 * race.  The default transform variant is used (no autotuning), and a
 * singular shifted system is not reported (it cannot arise for 0 < alpha < 1
 * when A has no eigenvalue with positive real part).  The first call on each
 * device looks up the array's address: make one call before capturing a
 * graph. */
#define CN_NOALLOC_SCRATCH_BYTES (64u << 20)
cn_status cn_pc_apply_noalloc(const cn_problem *p, const double *v, double *z);

/* Inspection of the last cycle's Arnoldi process (for tests; synchronises the
 * handle's stream).  The Gram-Schmidt step keeps the Gram matrix of the
 * normalised basis, G_pq = <v_p, v_q>/(||v_p|| ||v_q||), formed from the
 * stored vectors.  k: the inner iterations of the last cycle of the latest
 * cn_gmres_solve (its cn_gmres_info.iters when it did not restart; basis
 * vectors 0..k exist; CN_EINVAL outside [0, m_max]).  cn_aao_cycle returns G
 * (gram: (k+1)^2 doubles, row-major), the columns of the least-squares
 * triangular factor after the Givens rotations (rfac: k (k+1) doubles,
 * column j at j (k+1), rows 0..j) and the scales 1/||v_q|| of the stored,
 * unnormalised vectors (scale: k+1 doubles; scale[0] is overwritten by the
 * solve's final residual check and does not describe v_0).  Host arrays,
 * each may be NULL.  cn_aao_basis copies the stored basis vector q
 * (0 <= q <= m_max, unnormalised) into out (device, N_t N_x doubles, row
 * pitch N_x). */
cn_status cn_aao_cycle(cn_aao *h, int32_t k, double *gram, double *rfac, double *scale);
cn_status cn_aao_basis(cn_aao *h, int32_t q, double *out);

/* ---------------------------------------------------------------------------
 * Batches: many independent problems of uneven sizes solved together.  Every
 * step of the method (each transform, interface solve, matvec, Gram-Schmidt
 * pass, finishing reduction, update) is one kernel launch over a work list
 * covering all instances; instances that converged skip their work.  The
 * transform kernels run one launch per distinct N_t, with the (tile width,
 * workgroup size) variant chosen by the create-time autotuner on that
 * group's widest instance.
 * ------------------------------------------------------------------------- */
typedef struct cn_batch cn_batch;

/* Create a batch of `count` problems (each validated as by cn_aao_create).
 * All problems need the same pc_prec and stream.  Packed vectors hold the
 * instances back to back in order: instance i occupies [off[i], off[i+1])
 * of b and x (n_i = nx_i * nt_i elements), and [space_off[i], space_off[i+1])
 * of a packed u0 (nx_i elements).  Errors name the failing problem. */
cn_status cn_batch_create(const cn_problem *probs, int32_t count, cn_batch **out);
cn_status cn_batch_destroy(cn_batch *b);

/* Offsets of the packed layout: off and space_off are host arrays of
 * count+1 int64 (either may be NULL). */
cn_status cn_batch_offsets(const cn_batch *b, int64_t *off, int64_t *space_off);

/* Packed b = xi + tau f for every instance (u0 packed by space_off, f and b
 * packed by off); device pointers. */
cn_status cn_batch_rhs(cn_batch *b, const double *u0, const double *f, double *bp);

/* Solve every instance with GMRES(m) as cn_gmres_solve does (flexible form,
 * CGS2, float64 Krylov; preconditioner in the batch's precision).  opts->m
 * must not exceed the smallest m_max of the batch; the iteration budget
 * counts cycles' inner iterations of the batch as a whole.  infos: host array
 * of `count` entries (may be NULL); total (may be NULL) gets the largest
 * iteration count and relative residual and the summed matvecs.  Returns
 * CN_OK when every instance reached rtol, else CN_NOT_CONVERGED.
 * Synchronises. */
cn_status cn_batch_solve(cn_batch *b, const double *bp, double *xp, const cn_gmres_opts *opts,
                         cn_gmres_info *infos, cn_gmres_info *total);

/* Kernel timing of one inner iteration, for benchmarking.  Must follow a
 * cn_gmres_solve on the same handle that ran at least j+1 inner iterations
 * (its basis is reused; the solution is not touched).  Launches each of the
 * kernels of iteration j `reps` times back to back on the handle's
 * stream, timed with HIP events, and returns per kernel the average launch
 * duration in milliseconds and the algorithmic bytes one launch must move
 * (reads + writes of its inputs and outputs, each touched once).  Kernel
 * order: 0 pc_forward (steps (a) + local (b)), 1 pc_reduced (interface
 * systems of (b)), 2 pc_inverse (correction + step (c)), 3 matvec fused with
 * the dots against the basis, 4 Gram-Schmidt update (both projections, with
 * the reduction of the matvec's dots) + norm + Gram row of the new vector;
 * the one-workgroup Givens kernel is not included.  ms and bytes: host
 * arrays of CN_PROFILE_KERNELS doubles.  Synchronises. */
#define CN_PROFILE_KERNELS 5
cn_status cn_profile_step(cn_aao *h, int32_t j, int32_t reps, double *ms, double *bytes);

const char *cn_status_string(cn_status s);
const char *cn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CN_AAO_H */
