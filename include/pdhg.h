/*
 * libpdhg: restarted Halpern PDHG (r2HPDHG) for linear programs and restarted
 * accelerated PDHG (rAPDHG) for convex quadratic programs on AMD MI355X
 * (gfx950), behind a plain C ABI.
 *
 * Problem (MPAX paper, Section 2, eq. (qp)):
 *
 *     min  1/2 x'Qx + c'x   s.t.  l_c <= A x <= u_c,   l_v <= x <= u_v
 *
 * with A (m x n), Q (n x n, convex), Q = 0 for an LP. Absent bounds are
 * -INFINITY / +INFINITY. The solver works on the saddle form of eq.
 * (primal-dual-qp); y >= 0 on rows with only a lower bound, y <= 0 on rows with
 * only an upper bound, y free on two-sided rows.
 *
 * Conventions for every entry point below:
 *  - Types: int32_t for m, n and indices; int64_t for nnz and counters; double
 *    (FP64) for every value.
 *  - Errors are returned as pdhg_err; nothing aborts or throws across the ABI.
 *    pdhg_last_error() gives a message for the calling thread.
 *  - Solve outcomes (optimal, limits, numerical trouble) are reported in
 *    pdhg_result.status, separately from API errors.
 *  - The caller owns every buffer it passes; the library owns its scaled
 *    copies and workspace and frees them in pdhg_destroy / pdhg_batch_destroy.
 *  - Vector arguments of solve / step / scaling calls are DEVICE pointers on
 *    the GPU the handle was created on. Problem data handed to *_create may
 *    live on the host or the device (pdhg_problem.mem).
 *  - The library runs on a stream of its own. The caller's stream (passed to
 *    *_create as void*, a hipStream_t; NULL = the default stream) must outlive
 *    the handle: every call first waits for the work already queued on it, so
 *    inputs produced there are complete, and returns after its own GPU work
 *    has completed.
 *  - A handle must not be used from two threads at the same time.
 */
#ifndef PDHG_H
#define PDHG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PDHG_OK = 0,
    PDHG_ERR_INVALID_ARG = -1,   /* NULL pointer, negative size, bad option value */
    PDHG_ERR_INVALID_INPUT = -2, /* NaN / inf data, l > u, malformed CSR */
    PDHG_ERR_OOM = -3,           /* device allocation failed */
    PDHG_ERR_HIP = -4,           /* a HIP runtime call failed */
    PDHG_ERR_UNSUPPORTED = -5    /* valid but not supported combination */
} pdhg_err;

typedef enum {
    PDHG_UNSOLVED = 0,
    PDHG_OPTIMAL = 1,            /* relative KKT error <= eps */
    PDHG_PRIMAL_INFEASIBLE = 2,  /* a dual ray certifies that no x is feasible */
    PDHG_DUAL_INFEASIBLE = 3,    /* a primal ray certifies an unbounded objective */
    PDHG_ITERATION_LIMIT = 4,
    PDHG_TIME_LIMIT = 5,
    PDHG_NUMERICAL_ERROR = 6     /* NaN in the KKT terms */
} pdhg_status;

enum { PDHG_FMT_NONE = 0, PDHG_FMT_CSR = 1, PDHG_FMT_DENSE = 2, PDHG_FMT_LOWRANK_DIAG = 3 };
enum { PDHG_MEM_HOST = 0, PDHG_MEM_DEVICE = 1 };

/* Problem data (eq. (qp)). CSR matrices must have rowptr[0] = 0, non-decreasing
 * rowptr, rowptr[rows] = nnz, and strictly increasing column indices inside a
 * row; dense matrices are row-major. The library copies what it needs during
 * *_create; the caller may free the arrays afterwards. */
typedef struct {
    int32_t m, n;
    int32_t a_format;            /* PDHG_FMT_CSR or PDHG_FMT_DENSE */
    const int32_t *a_rowptr;     /* [m+1]  (CSR) */
    const int32_t *a_colidx;     /* [nnz]  (CSR) */
    const double *a_val;         /* [nnz]  (CSR) */
    int64_t a_nnz;               /* must equal a_rowptr[m] (CSR) */
    const double *a_dense;       /* [m*n]  (DENSE) */
    const double *c;             /* [n] objective */
    const double *lc, *uc;       /* [m] row bounds */
    const double *lv, *uv;       /* [n] variable bounds */
    int32_t q_format;            /* NONE, CSR, DENSE or LOWRANK_DIAG */
    const int32_t *q_rowptr;     /* [n+1]  (CSR) */
    const int32_t *q_colidx;     /* [q_nnz] (CSR) */
    const double *q_val;         /* [q_nnz] (CSR) */
    int64_t q_nnz;
    const double *q_dense;       /* [n*n]  (DENSE) */
    int32_t q_rank;              /* r (LOWRANK_DIAG): Q = F F' + diag(d) */
    const double *q_factor;      /* [n*r] row-major F (LOWRANK_DIAG) */
    const double *q_diag;        /* [n]   d (LOWRANK_DIAG) */
    int32_t mem;                 /* PDHG_MEM_HOST or PDHG_MEM_DEVICE for all arrays */
} pdhg_problem;

/* Options. Defaults (pdhg_options_default) follow the paper's Appendix A where
 * it gives a value (eps 1e-4, unlimited iterations, display every 10 checks)
 * and the documented readings elsewhere. */
typedef struct {
    double eps;                  /* relative KKT tolerance (eps_abs = eps_rel) */
    int64_t iteration_limit;     /* PDHG steps; INT64_MAX = none */
    double time_limit_s;         /* <= 0: none */
    int32_t check_every;         /* termination / restart cadence (iterations) */
    int32_t ruiz_iters;          /* Ruiz passes */
    int32_t pock_chambolle;      /* 1: one Pock-Chambolle (alpha = 1) pass */
    double gamma;                /* reflection coefficient in [0, 1] */
    double step_safety;          /* eta = step_safety / ||A~||_2 */
    double restart_sufficient;   /* 0.2 */
    double restart_necessary;    /* 0.8 */
    double restart_artificial;   /* 0.36 */
    double power_tol;            /* relative change stopping the norm estimates */
    int32_t power_max_iters;
    int32_t verbose;             /* 1: one line per display_frequency checks */
    int32_t display_frequency;   /* in checks */
    int32_t use_graph;           /* 1: replay each check period as a HIP graph */
    int32_t timing_chunk;        /* >= 0: time the iteration kernels of that
                                    check period with HIP events (result.kernel_*) */
    /* Infeasibility certificates (Appendix A: 1e-8 each; <= 0 switches the
     * test off). Tested at the checks of every solve (LP with CSR or dense
     * A, QP, single or batched) once a restart has happened: the rays are the PDHG
     * point (the averages for a QP) minus the restart anchor; a QP's primal
     * ray must also satisfy Q dx = 0. In a batch each instance stops on its
     * own certificate and its output slice holds the ray, as for pdhg_solve;
     * with both tolerances <= 0 the batched kernels skip the ray terms and
     * keep a smaller register budget. */
    double eps_primal_infeasible;
    double eps_dual_infeasible;
    /* Feasibility polishing (Section 3; Appendix A: off, 1e-6): after an
     * optimal LP solve, a primal phase (c = 0, from x) and a dual phase (the
     * finite bounds set to 0, from y) run to relative primal / dual
     * residuals <= eps_feas_polish; the solve returns x of the first and y
     * of the second, with the KKT terms of that point. */
    int32_t feasibility_polishing;
    double eps_feas_polish;
    /* Layouts of the iteration products of a large CSR constraint matrix
     * (the panels serve the checks' products with A~' too, the checks'
     * products with A~ keep the standard layout; results differ only in the
     * order of summation). -1 selects the automatic choice.
     * panel_rows: entries of y staged in LDS per panel for the product A~'y
     *   over the longest rows of A~' (auto: 20480 when m > 262144, else off;
     *   0: off; at most 20480);
     * panel_min_len: rows of A~' longer than this use the panels (auto: 32);
     * panel_wgs: workgroups per panel (auto: 12);
     * hot_cols: leading entries of x_ext staged in LDS by the product A~x_ext
     *   (auto: 20480 when n > 262144, else off; 0: off; at most 20480). */
    int32_t panel_rows;
    int32_t panel_min_len;
    int32_t panel_wgs;
    int32_t hot_cols;
} pdhg_options;

typedef struct {
    int32_t status;              /* pdhg_status */
    int64_t iterations;          /* PDHG steps taken */
    int64_t restarts;
    double primal_obj, dual_obj;
    double rel_primal_res, rel_dual_res, rel_gap, kkt_rel;
    double solve_seconds;        /* pdhg_solve wall time */
    double setup_seconds;        /* pdhg_create wall time (copied from the handle) */
    double eta, omega, norm_a, norm_q;
    int32_t power_iters;
    /* HIP-event timings of one check period (timing_chunk), milliseconds */
    int32_t kernel_samples;      /* number of timed plain iterations */
    double kernel_primal_ms;     /* average primal step: earliest start to latest end of its
                                    kernels (two streams when the LDS panels run) */
    double kernel_dual_ms;       /* average dual-step kernel duration */
    int64_t polish_iterations;   /* iterations of the polishing phases (in iterations too) */
} pdhg_result;

typedef struct pdhg_handle pdhg_handle;

void pdhg_options_default(pdhg_options *opt);

/* Message of the last error on the calling thread (never NULL). */
const char *pdhg_last_error(void);

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t pdhg_version(void);

/* Copy A (and Q) into library-owned device memory, apply the diagonal
 * preconditioning of Section 3 (Ruiz, then Pock-Chambolle), estimate
 * ||A~||_2 by Golub-Kahan-Lanczos bidiagonalisation (||Q~||_2 by power
 * iteration) and set the step size and the initial primal weight. stream: hipStream_t whose prior work the call waits
 * for (NULL = default stream). On success *out receives a handle that
 * pdhg_destroy releases. Errors: INVALID_ARG, INVALID_INPUT, OOM, HIP. */
pdhg_err pdhg_create(const pdhg_problem *prob, const pdhg_options *opt, void *stream,
                     pdhg_handle **out);

/* Run r2HPDHG (Algorithm 1; rAPDHG, Algorithm 2, when Q != 0) to the relative
 * KKT tolerance or a limit. x_init [n], y_init [m]: optional warm start in the
 * original space (NULL = zeros, Section 3 "Warm start"); it is scaled and
 * projected onto the bounds. x_out [n], y_out [m]: original-space solution
 * (the last PDHG point for LP, the weighted average for QP), written in every
 * outcome, except that on PDHG_PRIMAL_INFEASIBLE y_out holds the dual ray
 * D_r (yhat - y0) scaled to dual objective l_c'y+ - u_c'y- + l_v'lam+ -
 * u_v'lam- = 1 (lam the bound-cone part of -A'y), and on
 * PDHG_DUAL_INFEASIBLE x_out holds the primal ray D_c (xhat - x0) scaled to
 * c'x = -1. res may be NULL. All vector pointers are device pointers. */
pdhg_err pdhg_solve(pdhg_handle *h, const double *x_init, const double *y_init,
                    double *x_out, double *y_out, pdhg_result *res);

/* Replace c and the bounds of an existing handle (A, Q and the scaling stay);
 * device pointers, NULL keeps the current vector. The step size stays; the
 * initial primal weight is recomputed. */
pdhg_err pdhg_update_data(pdhg_handle *h, const double *c, const double *lc,
                          const double *uc, const double *lv, const double *uv);

/* Exactly one LP iteration (eq. (pdhg-lp) then eq. (hrpdhg)) in the SCALED
 * space, original variable order: from (x, y) with anchors (x0, y0), inner
 * counter k, steps tau, sigma, writes the PDHG point (xhat, yhat) and the
 * Halpern point (xnew, ynew). Uses the same kernels as pdhg_solve. Device
 * pointers; outputs may be NULL. LP handles only (UNSUPPORTED otherwise). */
pdhg_err pdhg_debug_step(pdhg_handle *h, const double *x, const double *y,
                         const double *x0, const double *y0, int64_t k, double tau,
                         double sigma, double *xhat, double *yhat, double *xnew,
                         double *ynew);

/* Exactly one plain LP iteration (eq. (pdhg-lp) then eq. (hrpdhg)), the one
 * that pdhg_solve runs between checks, in the SCALED space, original variable
 * order: from (x, y) with anchors (x0, y0), inner counter k and steps tau,
 * sigma, writes the Halpern point (xnew, ynew). It runs the kernels and
 * product layouts of the solve's plain iterations (the LDS panels and hot
 * columns of a large sparse A), which pdhg_debug_step (check kernels) does
 * not. Device pointers; outputs may be NULL. LP handles only (UNSUPPORTED
 * otherwise). */
pdhg_err pdhg_debug_plain_step(pdhg_handle *h, const double *x, const double *y,
                               const double *x0, const double *y0, int64_t k, double tau,
                               double sigma, double *xnew, double *ynew);

/* Exactly one rAPDHG iteration (Algorithm 2) in the SCALED space, original
 * variable order, for a handle with a quadratic term: from (x, y) and the
 * averages (xbar, ybar) with inner counter k and primal weight omega
 * (beta_k = theta_k = 2/(k+2), 1/tau_k = omega/eta + 2 ||Q~||_2/(k+1),
 * sigma = eta omega), writes the new iterate (xn, yn) and averages (xbarn,
 * ybarn). Device pointers; outputs may be NULL. UNSUPPORTED for LP handles. */
pdhg_err pdhg_debug_qp_step(pdhg_handle *h, const double *x, const double *y,
                            const double *xbar, const double *ybar, int64_t k, double omega,
                            double *xn, double *yn, double *xbarn, double *ybarn);

/* Scaling of Section 3 in the original order: D_r [m], D_c [n] (device
 * pointers, may be NULL) with A~ = D_r A D_c; scalars (host pointer to 4
 * doubles, may be NULL): eta, initial omega, ||A~||_2 estimate, ||Q~||_2
 * estimate; power_iters (host, may be NULL). */
pdhg_err pdhg_get_scaling(pdhg_handle *h, double *dr, double *dc, double *scalars,
                          int32_t *power_iters);

/* Release everything the handle owns. NULL is ignored. */
void pdhg_destroy(pdhg_handle *h);

/* ---------------------------------------------------------------------------
 * Batched LPs (Section 3, "Batched solving"): many independent LPs solved in
 * one persistent launch. Every instance runs its own r2HPDHG: own scaling
 * (shared when A is shared, since it depends on A only), step size, primal
 * weight, restarts and early exit, exactly as pdhg_solve would on that
 * instance alone.
 *
 * shared_a = 1: all B instances use one A (m x n, CSR); per-instance vectors
 *   are instance-major: c, lv, uv [B*n], lc, uc [B*m].
 * shared_a = 0 (ragged): instance b owns rows [row_off[b], row_off[b+1]) and
 *   columns [col_off[b], col_off[b+1]) of one block-diagonal CSR (m = total
 *   rows, n = total columns, global column indices that must stay inside the
 *   instance's column range); vectors are concatenated: c, lv, uv [n],
 *   lc, uc [m].
 */
typedef struct {
    int32_t batch;
    int32_t shared_a;
    int32_t m, n;
    const int32_t *a_rowptr;
    const int32_t *a_colidx;
    const double *a_val;
    int64_t a_nnz;
    const int32_t *row_off, *col_off;   /* [batch+1] (ragged only) */
    const double *c, *lc, *uc, *lv, *uv;
    /* Optional quadratic term (shared A only, rAPDHG): Q_b = F F' + diag(d_b)
     * with F [n*q_rank] row-major shared by the batch and d [B*n] per instance;
     * q_rank = 0 for LP batches, at most 32. */
    int32_t q_rank;
    const double *q_factor;
    const double *q_diag;
    int32_t mem;                        /* PDHG_MEM_HOST or PDHG_MEM_DEVICE */
} pdhg_batch_problem;

typedef struct pdhg_batch pdhg_batch;

/* Copy the batch, scale every instance and estimate its step size (one
 * persistent launch). iteration_limit must be finite (at most 10^7) so that
 * every workgroup of the persistent kernels ends. Errors as pdhg_create. */
pdhg_err pdhg_batch_create(const pdhg_batch_problem *prob, const pdhg_options *opt,
                           void *stream, pdhg_batch **out);

/* Solve all instances in one persistent launch. x_init / y_init: optional
 * warm starts laid out like c / lc (device pointers, may be NULL). x_out,
 * y_out: device pointers laid out like c / lc. res: HOST array of `batch`
 * results, may be NULL. */
pdhg_err pdhg_batch_solve(pdhg_batch *b, const double *x_init, const double *y_init,
                          double *x_out, double *y_out, pdhg_result *res);

/* Launch shape of the persistent kernels: threads per instance (64, 128,
 * 256, 512 or 1024) and the number of resident workgroups (<= 0: as many as
 * the GPU holds). The default after create is 1024 threads when the batch
 * has at most one instance per compute unit, else the fewest threads, from
 * 256, that give each thread at most 8 columns and 8 rows of the largest
 * instance; QP batches, and LP solves that test infeasibility rays, take at
 * most 512 of them unless this call or pdhg_batch_autotune chose the shape. */
pdhg_err pdhg_batch_set_launch(pdhg_batch *b, int32_t threads, int32_t workgroups);

/* Time `iterations` iterations of every instance for each supported thread
 * count and keep the fastest (written to *best_threads, may be NULL); for QP
 * batches the trials are batched rAPDHG solves limited to `iterations`. The
 * solver state is reset afterwards. */
pdhg_err pdhg_batch_autotune(pdhg_batch *b, int32_t iterations, int32_t *best_threads);

/* Replace the per-instance vectors (device pointers laid out as at create,
 * NULL keeps the current one). Scaling and step sizes stay (they depend on A
 * only); the initial primal weight is recomputed at the next solve. */
pdhg_err pdhg_batch_update_data(pdhg_batch *b, const double *c, const double *lc,
                                const double *uc, const double *lv, const double *uv);

/* Differentiation by unrolling (Section 3 "Auto-differentiation"): every
 * instance (LP or QP batch) runs exactly T iterations from zero with no
 * termination test. replay = 0: restart and primal-weight decisions come
 * from the regular tests and are recorded; replay = 1: the recorded schedule
 * of the last replay = 0 call with the same T is reused (so the map from c
 * and the row bounds to the output is piecewise affine and finite
 * differences through it are meaningful). The projection state of every
 * iteration is kept as bits for the reverse pass. x_out, y_out: the PDHG
 * point of iteration T-1 in the original space (device, laid out like c /
 * lc); for QP batches (rAPDHG) the averages (xbar, ybar) of iteration T-1.
 * T in [1, 10^6]. */
pdhg_err pdhg_batch_unrolled_forward(pdhg_batch *b, int64_t T, int32_t replay, double *x_out,
                                     double *y_out);

/* Reverse pass of the last unrolled forward: given cotangents gx (like c) and
 * gy (like lc, NULL = 0) of its outputs, writes the gradients with respect to
 * the original c (gc), row bounds (glc, guc; 0 for infinite bounds) and, for
 * QP batches, the diagonal d of Q (gd); NULL skips glc / guc / gd. Two sparse
 * products per reversed iteration. QP batches (rAPDHG, whose output is the
 * average) keep the state every 50 iterations during the forward pass and
 * recompute each segment to get the momentum points. Device pointers. */
pdhg_err pdhg_batch_unrolled_backward(pdhg_batch *b, const double *gx, const double *gy,
                                      double *gc, double *glc, double *guc, double *gd);

/* Release everything the batch owns. NULL is ignored. */
void pdhg_batch_destroy(pdhg_batch *b);

/* ---- Loss heads of the end-to-end learning pipelines (Section 4: the
 * shortest-path experiment with a regret loss, and differentiating QP
 * solutions). Device pointers, work enqueued on `stream` (a hipStream_t, NULL
 * = default stream); the functions return once the work is enqueued, except
 * pdhg_linear_costs_backward, which also waits for it. Sums are deterministic
 * (fixed-order workgroup trees). Errors: PDHG_ERR_INVALID_ARG for bad sizes
 * or NULL arrays. ---- */

/* Linear cost model on features: c_hat[i] = sum_k W[k] f[i p + k] for the
 * N = B n variables (f row-major [B n][p], 1 <= p <= 64). */
pdhg_err pdhg_linear_costs(int32_t B, int32_t n, int32_t p, const double *f, const double *W,
                           double *c_hat, void *stream);

/* Regret of decisions x [B n] under the true costs: loss[b] = c_true_b' x_b
 * - v_star[b], v_star the optimal value under c_true. Its gradient in x_b is
 * c_true_b, the cotangent to hand to pdhg_batch_unrolled_backward. */
pdhg_err pdhg_regret(int32_t B, int32_t n, const double *c_true, const double *x,
                     const double *v_star, double *loss, void *stream);

/* Weight gradient of the linear cost model: gW[k] = sum_i gc[i] f[i p + k]
 * for a cotangent gc [B n] of c_hat (e.g. the gc of the unrolled reverse
 * pass). gW has p entries. */
pdhg_err pdhg_linear_costs_backward(int32_t B, int32_t n, int32_t p, const double *f,
                                    const double *gc, double *gW, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same weight
 * gradient as pdhg_linear_costs_backward, bit for bit, with its partial sums
 * in a static 32 KB device array (64 x 64 doubles, one per GPU, held until the
 * process ends) instead of a buffer allocated per call. It allocates nothing
 * and returns once the work is enqueued on `stream` (no wait). Limit: p <= 64
 * (PDHG_ERR_INVALID_ARG beyond). Every call on one GPU uses that GPU's array,
 * so calls that overlap on a GPU (other threads or streams) race and must be
 * ordered by the caller. */
pdhg_err pdhg_linear_costs_backward_noalloc(int32_t B, int32_t n, int32_t p, const double *f,
                                            const double *gc, double *gW, void *stream);

/* Objective value of B QPs with Q_b = F F' + diag(d_b) (F [n r] row-major,
 * shared, r <= 32; d, c, x [B n]): value[b] = 1/2 x_b' Q_b x_b + c_b' x_b and,
 * when gx is not NULL, its gradient gx_b = Q_b x_b + c_b. */
pdhg_err pdhg_qp_value(int32_t B, int32_t n, int32_t r, const double *F, const double *d,
                       const double *c, const double *x, double *value, double *gx,
                       void *stream);

/* ---- Surrogate losses for LP (Section 3.4 names SPO+ and the perturbed
 * Fenchel-Young loss; Section 4.4 trains with SPO+). Both are stated for
 * min_{w in S} c'w over the LP's feasible set S; the optimal solutions they
 * take come from pdhg_batch_solve. Layouts as above ([B n] row-major,
 * device pointers, work enqueued on `stream`). ---- */

/* Costs of the SPO+ inner problem: c_out = 2 c_hat - c_true ([B n]). */
pdhg_err pdhg_spo_plus_costs(int32_t B, int32_t n, const double *c_hat, const double *c_true,
                             double *c_out, void *stream);

/* SPO+ loss and subgradient. w_star [B n] is optimal under c_true with
 * value z_star [B]; w_tilde [B n] is optimal under 2 c_hat - c_true. Then
 * loss[b] = -(2 c_hat_b - c_true_b)'w_tilde_b + 2 c_hat_b'w_star_b - z_star[b]
 * and grad_b = 2 (w_star_b - w_tilde_b), a subgradient in c_hat_b. */
pdhg_err pdhg_spo_plus(int32_t B, int32_t n, const double *c_hat, const double *c_true,
                       const double *w_star, const double *z_star, const double *w_tilde, double *loss,
                       double *grad, void *stream);

/* Perturbed costs of the Fenchel-Young estimator: c_out [B M n], sample
 * (b, m) = c_hat_b + eps Z_bm for the caller's draws Z [B M n] (standard
 * normal); M >= 1, eps finite. */
pdhg_err pdhg_pfy_costs(int32_t B, int32_t M, int32_t n, const double *c_hat, const double *Z, double eps,
                        double *c_out, void *stream);

/* Perturbed Fenchel-Young loss (up to the constant Omega(w_star), which does
 * not depend on c_hat) and gradient from M samples: w_samples [B M n] optimal
 * under the costs of pdhg_pfy_costs; loss[b] = c_hat_b'w_star_b - (1/M)
 * sum_m (c_hat_b + eps Z_bm)'w_bm, grad_b = w_star_b - (1/M) sum_m w_bm. */
pdhg_err pdhg_pfy(int32_t B, int32_t M, int32_t n, const double *c_hat, const double *w_star,
                  const double *Z, double eps, const double *w_samples, double *loss, double *grad,
                  void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PDHG_H */
