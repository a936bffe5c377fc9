/*
 * Plain FP64 CPU oracle for restarted Halpern PDHG (LP) and restarted
 * accelerated PDHG (QP).
 *
 * TEST INFRASTRUCTURE ONLY. This code is the independent reference that the
 * GPU library is checked against. Only the test suite, the package smoke test
 * and the benchmark's CPU-baseline leg may load it. The GPU library shares no
 * code, header or constant with it.
 *
 * Problem (paper, Section 2, eq. (qp)):
 *     min 1/2 x'Qx + c'x   s.t.  l_c <= A x <= u_c,  l_v <= x <= u_v
 * with +-inf marking absent bounds. Dot products and norms accumulate in
 * long double. Nothing is blocked, fused or reordered beyond the equations.
 *
 * Parity status of each part is documented next to each function in oracle.c.
 */
#ifndef PDHG_ORACLE_H
#define PDHG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t m, n;
    /* constraint matrix: CSR (rowptr/colidx/val) or dense row-major (dense) */
    const int32_t *rowptr, *colidx;
    const double *val;
    const double *dense;
    const double *c, *lc, *uc, *lv, *uv;
    /* quadratic term: 0 none, 1 CSR (q_rowptr/q_colidx/q_val),
     * 2 low rank + diagonal, Q = F F' + diag(d) with F n x r row-major */
    int32_t q_kind;
    const int32_t *q_rowptr, *q_colidx;
    const double *q_val;
    int32_t q_rank;
    const double *q_factor, *q_diag;
} orc_problem;

typedef struct {
    double eps;                 /* relative KKT tolerance */
    int64_t iteration_limit;
    int32_t check_every;
    int32_t ruiz_iters;
    int32_t pock_chambolle;     /* 1: one Pock-Chambolle alpha=1 step */
    double gamma;               /* reflection coefficient */
    double step_safety;         /* eta = step_safety / ||A~||_2 */
    double restart_sufficient, restart_necessary, restart_artificial;
    double power_tol;
    int32_t power_max_iters;
    int32_t verbose;
    /* certificate tolerances of the infeasibility tests (<= 0: off) */
    double eps_primal_infeasible, eps_dual_infeasible;
    /* 1: polish the point of an optimal LP solve to eps_feas_polish */
    int32_t feasibility_polishing;
    double eps_feas_polish;
} orc_options;

typedef struct {
    int32_t status;             /* 1 optimal, 2 primal infeasible, 3 dual infeasible,
                                   4 iteration limit, 6 numerical error */
    int64_t iterations, restarts;
    double primal_obj, dual_obj;
    double rel_primal, rel_dual, rel_gap, kkt;
    double abs_primal, abs_dual, abs_gap;  /* ||r_p||, ||r_d||, |P - D| */
    double eta, omega, norm_a, norm_q;
    int32_t power_iters;
    int64_t polish_iterations;  /* iterations of the two polishing phases */
} orc_result;

typedef struct orc_ctx orc_ctx;

void orc_default_options(orc_options *o);

/* Scale the problem and estimate the step size. Returns NULL on invalid input. */
orc_ctx *orc_create(const orc_problem *p, const orc_options *o);
int orc_threads(void);          /* threads the products use (0 without OpenMP) */
void orc_set_threads(int t);    /* t > 0: threads for the products */
void orc_destroy(orc_ctx *ctx);

/* Scaling vectors D_r [m], D_c [n]; step eta, initial primal weight omega,
 * ||A~||_2 and ||Q~||_2 estimates. */
void orc_scaling(const orc_ctx *ctx, double *dr, double *dc, double *eta,
                 double *omega, double *norm_a, double *norm_q, int32_t *power_iters);

/* Pin the step-size constants (eta, ||Q~||_2) to given values, e.g. those of
 * a base problem, so that an unrolled run with perturbed data follows the
 * same frozen map. */
void orc_pin_steps(orc_ctx *ctx, double eta, double norm_q);

/* Scaled data: c~ [n], l~_c u~_c [m], l~_v u~_v [n]. */
void orc_scaled_vectors(const orc_ctx *ctx, double *c, double *lc, double *uc,
                        double *lv, double *uv);

/* One r2HPDHG iteration in the scaled space from state (x, y), anchors
 * (x0, y0), inner counter k, steps tau, sigma and reflection gamma.
 * Outputs the PDHG point (xhat, yhat) and the Halpern point (xnew, ynew).
 * Any output pointer may be NULL. */
void orc_lp_step(const orc_ctx *ctx, const double *x, const double *y,
                 const double *x0, const double *y0, int64_t k, double tau,
                 double sigma, double gamma, double *xhat, double *yhat,
                 double *xnew, double *ynew);

/* One rAPDHG iteration in the scaled space (momentum, averaging). */
void orc_qp_step(const orc_ctx *ctx, const double *x, const double *y,
                 const double *xbar, const double *ybar, int64_t k, double omega,
                 double *xn, double *yn, double *xbarn, double *ybarn);

/* Fixed-point residual of (x, y) -> (xhat, yhat) in the PDHG norm. */
double orc_fixed_point_residual(const orc_ctx *ctx, const double *x, const double *y,
                                const double *xhat, const double *yhat,
                                double tau, double sigma);

/* Relative KKT error of an original-space pair (x, y). */
void orc_kkt(const orc_problem *p, const double *x, const double *y, orc_result *r);

/* Full solve. x_init / y_init are original-space warm starts or NULL.
 * Writes the original-space solution into x_out [n], y_out [m]. */
int orc_solve(orc_ctx *ctx, const double *x_init, const double *y_init,
              double *x_out, double *y_out, orc_result *res);

/* Unrolled LP forward with a frozen schedule: exactly T iterations, no
 * early stop. The restart/primal-weight decisions are those of the regular
 * solver run on the same data (recorded internally) unless
 * sched_* are given: sched_restart[t] (1 = restart at iteration t) and
 * sched_omega[t] (primal weight used at iteration t). The final output is
 * the PDHG point of iteration T-1, unscaled. */
int orc_unrolled_lp(orc_ctx *ctx, int64_t T, const uint8_t *sched_restart,
                    const double *sched_omega, uint8_t *rec_restart,
                    double *rec_omega, double *x_out, double *y_out);

/* Reverse mode of orc_unrolled_lp with the same schedule: given cotangents
 * of the original-space outputs, returns gradients with respect to the
 * original c, l_c and u_c (entries for infinite bounds are 0). */
int orc_unrolled_lp_backward(orc_ctx *ctx, int64_t T, const uint8_t *sched_restart,
                             const double *sched_omega, const double *gx,
                             const double *gy, double *gc, double *glc, double *guc);

/* Unrolled rAPDHG (Algorithm 2) with a frozen schedule: exactly T iterations
 * from zero; restarts / weights from the tests (recorded) or from sched_*.
 * Output: the unscaled averages (xbar, ybar) after iteration T-1. */
int orc_unrolled_qp(orc_ctx *ctx, int64_t T, const uint8_t *sched_restart,
                    const double *sched_omega, uint8_t *rec_restart, double *rec_omega,
                    double *x_out, double *y_out);

/* Reverse pass of orc_unrolled_qp: gradients with respect to the original c,
 * l_c, u_c and the diagonal d of Q (low-rank + diagonal Q only; gd may be
 * NULL otherwise). */
int orc_unrolled_qp_backward(orc_ctx *ctx, int64_t T, const uint8_t *sched_restart,
                             const double *sched_omega, const double *gx, const double *gy,
                             double *gc, double *glc, double *guc, double *gd);

#ifdef __cplusplus
}
#endif
#endif
