/*
 * Plain FP64 CPU oracle for restarted Halpern PDHG (LP, Algorithm 1) and
 * restarted accelerated PDHG (QP, Algorithm 2) of "MPAX: Mathematical
 * Programming in JAX" (arXiv 2412.09734).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke test and the
 * benchmark's CPU-baseline leg, never by the GPU library.
 *
 * Every loop below follows one equation of the paper or one written reading of
 * a point the paper leaves open (the readings are listed in the design notes
 * with the same names used here: scaling, step size, primal weight, restart
 * rule, KKT composition, check cadence, rAPDHG schedule, frozen schedule).
 * Sums accumulate in long double; nothing is blocked or fused.
 *
 * The products with A~ and A~' may run on several threads (OpenMP over output
 * rows, or over columns through a column-major copy of A~): every output entry
 * is still summed alone, in the same order as on one thread, so results do not
 * depend on the thread count. All other loops, reductions included, are serial.
 *
 * Parity unpinned: restart_due (restart rule) and new_weight (primal-weight
 * update). The paper defers both rules to other solvers, so no value, closed
 * form or bound of its own pins them; only the final optima the oracle reaches
 * through them are pinned.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;

struct orc_ctx {
    orc_problem p;       /* original data (caller-owned pointers) */
    orc_options o;
    int32_t m, n;
    /* scaled constraint matrix: same layout as the input */
    double *val;         /* CSR values (nnz) or dense (m*n) */
    int dense;
    /* column-major copy of the scaled sparse A~ (rows ascending in a column) */
    int32_t *cptr, *crow;
    double *cval;
    /* scaled quadratic term */
    double *qval;        /* CSR values */
    double *qf;          /* n x r */
    double *qd;          /* n */
    double *dr, *dc;     /* D_r [m], D_c [n] */
    double *c, *lc, *uc, *lv, *uv;   /* scaled data */
    double eta, omega0, norm_a, norm_q;
    int32_t power_iters;
    int polish;          /* 0 solve; 1 / 2 primal / dual polishing phase */
};

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */

static double clampd(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }

static ld sumsq(const double *v, int32_t len) {
    ld s = 0.0L;
    for (int32_t i = 0; i < len; ++i) s += (ld)v[i] * (ld)v[i];
    return s;
}

static ld dot(const double *a, const double *b, int32_t len) {
    ld s = 0.0L;
    for (int32_t i = 0; i < len; ++i) s += (ld)a[i] * (ld)b[i];
    return s;
}

static double *dalloc(size_t len) {
    double *p = (double *)calloc(len ? len : 1, sizeof(double));
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

static ld *lalloc(size_t len) {
    ld *p = (ld *)calloc(len ? len : 1, sizeof(ld));
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

void orc_default_options(orc_options *o) {
    o->eps = 1e-4;                 /* eps_abs = eps_rel = 1e-4, Appendix A */
    o->iteration_limit = INT64_MAX;
    o->check_every = 64;
    o->ruiz_iters = 10;
    o->pock_chambolle = 1;
    o->gamma = 1.0;                /* Algorithm 1 uses 2 xhat - x */
    o->step_safety = 0.998;
    o->restart_sufficient = 0.2;
    o->restart_necessary = 0.8;
    o->restart_artificial = 0.36;
    o->power_tol = 1e-7;
    o->power_max_iters = 2000;
    o->verbose = 0;
    o->eps_primal_infeasible = 1e-8;   /* Appendix A */
    o->eps_dual_infeasible = 1e-8;
    o->feasibility_polishing = 0;      /* Appendix A: off, tolerance 1e-6 */
    o->eps_feas_polish = 1e-6;
}

/* ------------------------------------------------------------------------ */
/* products with the scaled matrices                                         */

/* out = A~ v  (m-vector) */
static void a_mul(const orc_ctx *s, const double *v, double *out) {
    const int32_t m = s->m, n = s->n;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < m; ++i) {
        ld acc = 0.0L;
        if (s->dense) {
            const double *row = s->val + (size_t)i * n;
            for (int32_t j = 0; j < n; ++j) acc += (ld)row[j] * (ld)v[j];
        } else {
            for (int32_t e = s->p.rowptr[i]; e < s->p.rowptr[i + 1]; ++e)
                acc += (ld)s->val[e] * (ld)v[s->p.colidx[e]];
        }
        out[i] = (double)acc;
    }
}

/* out = A~' w  (n-vector): entries of each column summed in row order */
static void at_mul(const orc_ctx *s, const double *w, double *out) {
    const int32_t m = s->m, n = s->n;
    if (s->cptr) {   /* the same sums, one column at a time */
#pragma omp parallel for schedule(static)
        for (int32_t j = 0; j < n; ++j) {
            ld acc = 0.0L;
            for (int32_t e = s->cptr[j]; e < s->cptr[j + 1]; ++e) acc += (ld)s->cval[e] * (ld)w[s->crow[e]];
            out[j] = (double)acc;
        }
        return;
    }
    ld *acc = lalloc(n);
    for (int32_t i = 0; i < m; ++i) {
        if (s->dense) {
            const double *row = s->val + (size_t)i * n;
            for (int32_t j = 0; j < n; ++j) acc[j] += (ld)row[j] * (ld)w[i];
        } else {
            for (int32_t e = s->p.rowptr[i]; e < s->p.rowptr[i + 1]; ++e)
                acc[s->p.colidx[e]] += (ld)s->val[e] * (ld)w[i];
        }
    }
    for (int32_t j = 0; j < n; ++j) out[j] = (double)acc[j];
    free(acc);
}

/* out = Q~ v (zero when there is no quadratic term) */
static void q_mul(const orc_ctx *s, const double *v, double *out) {
    const int32_t n = s->n;
    if (s->p.q_kind == 1) {
        for (int32_t k = 0; k < n; ++k) {
            ld acc = 0.0L;
            for (int32_t e = s->p.q_rowptr[k]; e < s->p.q_rowptr[k + 1]; ++e)
                acc += (ld)s->qval[e] * (ld)v[s->p.q_colidx[e]];
            out[k] = (double)acc;
        }
    } else if (s->p.q_kind == 2) {
        const int32_t r = s->p.q_rank;
        ld *t = lalloc(r);
        for (int32_t j = 0; j < n; ++j)
            for (int32_t q = 0; q < r; ++q) t[q] += (ld)s->qf[(size_t)j * r + q] * (ld)v[j];
        double *td = dalloc(r);
        for (int32_t q = 0; q < r; ++q) td[q] = (double)t[q];
        for (int32_t j = 0; j < n; ++j) {
            ld acc = 0.0L;
            for (int32_t q = 0; q < r; ++q) acc += (ld)s->qf[(size_t)j * r + q] * (ld)td[q];
            acc += (ld)s->qd[j] * (ld)v[j];
            out[j] = (double)acc;
        }
        free(t);
        free(td);
    } else {
        for (int32_t k = 0; k < n; ++k) out[k] = 0.0;
    }
}

/* out = Q v with the ORIGINAL quadratic term (for the KKT error) */
static void q_mul_orig(const orc_problem *p, const double *v, double *out) {
    const int32_t n = p->n;
    if (p->q_kind == 1) {
        for (int32_t k = 0; k < n; ++k) {
            ld acc = 0.0L;
            for (int32_t e = p->q_rowptr[k]; e < p->q_rowptr[k + 1]; ++e)
                acc += (ld)p->q_val[e] * (ld)v[p->q_colidx[e]];
            out[k] = (double)acc;
        }
    } else if (p->q_kind == 2) {
        const int32_t r = p->q_rank;
        ld *t = lalloc(r);
        for (int32_t j = 0; j < n; ++j)
            for (int32_t q = 0; q < r; ++q) t[q] += (ld)p->q_factor[(size_t)j * r + q] * (ld)v[j];
        for (int32_t j = 0; j < n; ++j) {
            ld acc = 0.0L;
            for (int32_t q = 0; q < r; ++q) acc += (ld)p->q_factor[(size_t)j * r + q] * t[q];
            acc += (ld)p->q_diag[j] * (ld)v[j];
            out[j] = (double)acc;
        }
        free(t);
    } else {
        for (int32_t k = 0; k < n; ++k) out[k] = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* validation                                                               */

static int validate(const orc_problem *p) {
    if (p->m < 0 || p->n < 1) return 0;
    if (!p->c || !p->lv || !p->uv) return 0;
    if (p->m > 0 && (!p->lc || !p->uc)) return 0;
    if (!p->dense) {
        if (!p->rowptr || p->rowptr[0] != 0) return 0;
        for (int32_t i = 0; i < p->m; ++i) {
            if (p->rowptr[i + 1] < p->rowptr[i]) return 0;
            for (int32_t e = p->rowptr[i]; e < p->rowptr[i + 1]; ++e) {
                int32_t j = p->colidx[e];
                if (j < 0 || j >= p->n) return 0;
                if (e > p->rowptr[i] && j <= p->colidx[e - 1]) return 0;
                if (!isfinite(p->val[e])) return 0;
            }
        }
    } else {
        for (size_t e = 0; e < (size_t)p->m * p->n; ++e)
            if (!isfinite(p->dense[e])) return 0;
    }
    for (int32_t j = 0; j < p->n; ++j) {
        if (!isfinite(p->c[j])) return 0;
        if (isnan(p->lv[j]) || isnan(p->uv[j]) || p->lv[j] > p->uv[j]) return 0;
        if (p->lv[j] == INFINITY || p->uv[j] == -INFINITY) return 0;
    }
    for (int32_t i = 0; i < p->m; ++i) {
        if (isnan(p->lc[i]) || isnan(p->uc[i]) || p->lc[i] > p->uc[i]) return 0;
        if (p->lc[i] == INFINITY || p->uc[i] == -INFINITY) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* preconditioning (Section 3: Ruiz, then Pock-Chambolle)                   */

/* Apply row factors r and column factors s to the scaled copy:
 * A~_ij <- A~_ij / (r_i s_j), D_r <- D_r / r, D_c <- D_c / s. */
static void apply_factors(orc_ctx *s, const double *r, const double *cs) {
    const int32_t m = s->m, n = s->n;
    for (int32_t i = 0; i < m; ++i) {
        if (s->dense) {
            double *row = s->val + (size_t)i * n;
            for (int32_t j = 0; j < n; ++j) row[j] = row[j] / (r[i] * cs[j]);
        } else {
            for (int32_t e = s->p.rowptr[i]; e < s->p.rowptr[i + 1]; ++e)
                s->val[e] = s->val[e] / (r[i] * cs[s->p.colidx[e]]);
        }
        s->dr[i] = s->dr[i] / r[i];
    }
    for (int32_t j = 0; j < n; ++j) s->dc[j] = s->dc[j] / cs[j];
}

/* Ruiz equilibration: each pass divides row i by sqrt(max_j |A~_ij|) and
 * column j by sqrt(max_i |A~_ij|) (both taken before the pass; a zero norm
 * gives factor 1). Pock-Chambolle with alpha = 1: same with 1-norms. */
static void scale(orc_ctx *s) {
    const int32_t m = s->m, n = s->n;
    double *r = dalloc(m), *cs = dalloc(n);
    for (int32_t pass = 0; pass < s->o.ruiz_iters + (s->o.pock_chambolle ? 1 : 0); ++pass) {
        const int pc = pass >= s->o.ruiz_iters;
        ld *rn = lalloc(m), *cn = lalloc(n);
        for (int32_t i = 0; i < m; ++i) {
            if (s->dense) {
                const double *row = s->val + (size_t)i * n;
                for (int32_t j = 0; j < n; ++j) {
                    ld a = fabsl((ld)row[j]);
                    if (pc) { rn[i] += a; cn[j] += a; }
                    else { if (a > rn[i]) rn[i] = a; if (a > cn[j]) cn[j] = a; }
                }
            } else {
                for (int32_t e = s->p.rowptr[i]; e < s->p.rowptr[i + 1]; ++e) {
                    int32_t j = s->p.colidx[e];
                    ld a = fabsl((ld)s->val[e]);
                    if (pc) { rn[i] += a; cn[j] += a; }
                    else { if (a > rn[i]) rn[i] = a; if (a > cn[j]) cn[j] = a; }
                }
            }
        }
        for (int32_t i = 0; i < m; ++i) {
            double v = (double)rn[i];
            r[i] = v > 0.0 ? sqrt(v) : 1.0;
        }
        for (int32_t j = 0; j < n; ++j) {
            double v = (double)cn[j];
            cs[j] = v > 0.0 ? sqrt(v) : 1.0;
        }
        apply_factors(s, r, cs);
        free(rn);
        free(cn);
    }
    free(r);
    free(cs);
}

/* ------------------------------------------------------------------------ */
/* power iteration for ||A~||_2 and ||Q~||_2                                 */

/* SplitMix64 (Steele, Lea and Flood, 2014): output for counter x. */
static uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Start vector of the power iterations: v_j = 0.5 + u_j, u_j uniform in
 * [0, 1) from SplitMix64 at counter j, scaled to unit length. (A constant
 * start vector can lie in the null space, e.g. for node-arc incidence
 * matrices, whose rows sum to zero.) */
static void start_vector(double *v, int32_t n) {
    for (int32_t j = 0; j < n; ++j)
        v[j] = 0.5 + (double)(splitmix64((uint64_t)j) >> 11) * 0x1.0p-53;
    double nv = (double)sqrtl(sumsq(v, n));
    for (int32_t j = 0; j < n; ++j) v[j] = v[j] / nv;
}

/* Largest eigenvalue of the k x k symmetric tridiagonal matrix T = B'B of the
 * Golub-Kahan bidiagonal B (alpha_1..alpha_k on the diagonal, beta_1..beta_{k-1}
 * above it): T_ii = alpha_i^2 + beta_{i-1}^2, T_i,i+1 = alpha_i beta_i. Bisection
 * on the Sturm count (number of eigenvalues below x) over [0, Gershgorin
 * bound] until the interval cannot be halved. */
static int sturm_below(const double *alpha, const double *beta, int32_t k, double x) {
    int cnt = 0;
    double q = 1.0;
    for (int32_t i = 0; i < k; ++i) {
        const double di = alpha[i] * alpha[i] + (i > 0 ? beta[i - 1] * beta[i - 1] : 0.0);
        if (i == 0) {
            q = di - x;
        } else {
            const double ei = alpha[i - 1] * beta[i - 1];
            q = di - x - (ei * ei) / q;
        }
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

static double tridiag_max(const double *alpha, const double *beta, int32_t k) {
    double hi = 0.0;
    for (int32_t i = 0; i < k; ++i) {
        const double di = alpha[i] * alpha[i] + (i > 0 ? beta[i - 1] * beta[i - 1] : 0.0);
        const double el = i > 0 ? fabs(alpha[i - 1] * beta[i - 1]) : 0.0;
        const double er = i + 1 < k ? fabs(alpha[i] * beta[i]) : 0.0;
        if (di + el + er > hi) hi = di + el + er;
    }
    double lo = 0.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (sturm_below(alpha, beta, k, mid) == k) hi = mid;
        else lo = mid;
    }
    return hi;
}

/* ||A~||_2 by Golub-Kahan-Lanczos bidiagonalisation from the start vector:
 *   p = A~ v_k - beta_{k-1} u_{k-1},  alpha_k = |p|,  u_k = p / alpha_k
 *   q = A~' u_k - alpha_k v_k,        beta_k = |q|,   v_{k+1} = q / beta_k
 * lam_k = largest eigenvalue of B_k'B_k (the square of the largest Ritz value
 * of A~); stop at the first k >= 2 with |lam_k - lam_{k-1}| <= tol lam_k, or
 * when the Krylov space closes (alpha or beta zero). Returns sqrt(lam). */
static double power_norm_a(const orc_ctx *s, int32_t *iters) {
    const int32_t m = s->m, n = s->n;
    const size_t nv = s->dense ? (size_t)m * n : (m > 0 ? (size_t)s->p.rowptr[m] : 0);
    if (m == 0 || nv == 0) {   /* no constraint entries: ||A~|| = 0, no steps */
        if (iters) *iters = 0;
        return 0.0;
    }
    const int32_t maxit = s->o.power_max_iters;
    double *v = dalloc(n), *u = dalloc(m), *uprev = dalloc(m), *p = dalloc(m), *q = dalloc(n);
    double *alpha = dalloc(maxit + 1), *beta = dalloc(maxit + 1);
    start_vector(v, n);
    for (int32_t i = 0; i < m; ++i) uprev[i] = 0.0;
    double lam = 0.0, lam_prev = 0.0, bprev = 0.0;
    int32_t it = 0;
    for (it = 1; it <= maxit; ++it) {
        a_mul(s, v, p);
        for (int32_t i = 0; i < m; ++i) p[i] = p[i] - bprev * uprev[i];
        const double a = (double)sqrtl(sumsq(p, m));
        if (!(a > 0.0)) { if (it == 1) lam = 0.0; break; }
        for (int32_t i = 0; i < m; ++i) { u[i] = p[i] / a; uprev[i] = u[i]; }
        at_mul(s, u, q);
        for (int32_t j = 0; j < n; ++j) q[j] = q[j] - a * v[j];
        const double b = (double)sqrtl(sumsq(q, n));
        alpha[it - 1] = a;
        beta[it - 1] = b;
        lam = tridiag_max(alpha, beta, it);
        if (!(b > 0.0)) break;
        if (it > 1 && fabs(lam - lam_prev) <= s->o.power_tol * lam) break;
        lam_prev = lam;
        for (int32_t j = 0; j < n; ++j) v[j] = q[j] / b;
        bprev = b;
    }
    if (it > maxit) it = maxit;
    if (iters) *iters = it;
    free(v); free(u); free(uprev); free(p); free(q); free(alpha); free(beta);
    return sqrt(lam);
}

static double power_norm_q(const orc_ctx *s) {
    const int32_t n = s->n;
    if (s->p.q_kind == 0) return 0.0;
    double *v = dalloc(n), *w = dalloc(n);
    start_vector(v, n);
    double lam = 0.0, lam_prev = 0.0;
    for (int32_t it = 1; it <= s->o.power_max_iters; ++it) {
        q_mul(s, v, w);
        lam = (double)dot(v, w, n);
        double nw = sqrtl(sumsq(w, n));
        if (!(nw > 0.0)) { lam = 0.0; break; }
        for (int32_t j = 0; j < n; ++j) v[j] = w[j] / nw;
        if (it > 1 && fabs(lam - lam_prev) <= s->o.power_tol * fabs(lam)) break;
        lam_prev = lam;
    }
    free(v); free(w);
    return lam;
}

/* ------------------------------------------------------------------------ */
/* setup                                                                     */

/* Transformed data of the current original vectors s->p: c~ = D_c c,
 * l~_c = D_r l_c, l~_v = l_v / D_c, and the initial primal weight
 * ||c~|| / ||b~|| (b~_i the largest finite |bound| of row i). */
static void set_vectors(orc_ctx *s) {
    const orc_problem *p = &s->p;
    const int32_t m = s->m, n = s->n;
    for (int32_t j = 0; j < n; ++j) {
        s->c[j] = s->dc[j] * p->c[j];
        s->lv[j] = p->lv[j] / s->dc[j];
        s->uv[j] = p->uv[j] / s->dc[j];
    }
    for (int32_t i = 0; i < m; ++i) {
        s->lc[i] = s->dr[i] * p->lc[i];
        s->uc[i] = s->dr[i] * p->uc[i];
    }
    double *bt = dalloc(m);
    for (int32_t i = 0; i < m; ++i) {
        double b = 0.0;
        if (isfinite(s->lc[i])) b = fmax(b, fabs(s->lc[i]));
        if (isfinite(s->uc[i])) b = fmax(b, fabs(s->uc[i]));
        bt[i] = b;
    }
    double cn = (double)sqrtl(sumsq(s->c, n)), bn = (double)sqrtl(sumsq(bt, m));
    s->omega0 = (cn > 1e-10 && bn > 1e-10) ? cn / bn : 1.0;
    free(bt);
}

orc_ctx *orc_create(const orc_problem *p, const orc_options *o) {
    if (!validate(p)) return NULL;
    orc_ctx *s = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    s->p = *p;
    s->o = *o;
    s->m = p->m;
    s->n = p->n;
    const int32_t m = p->m, n = p->n;
    s->dense = p->dense != NULL;
    size_t nv = s->dense ? (size_t)m * n : (size_t)p->rowptr[m];
    s->val = dalloc(nv);
    memcpy(s->val, s->dense ? p->dense : p->val, nv * sizeof(double));
    s->dr = dalloc(m);
    s->dc = dalloc(n);
    for (int32_t i = 0; i < m; ++i) s->dr[i] = 1.0;
    for (int32_t j = 0; j < n; ++j) s->dc[j] = 1.0;
    scale(s);
    if (!s->dense && m > 0) {   /* column-major copy of A~: rows ascending within a column */
        const int32_t nnz = p->rowptr[m];
        s->cptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
        s->crow = (int32_t *)malloc(sizeof(int32_t) * (nnz > 0 ? nnz : 1));
        s->cval = dalloc(nnz > 0 ? nnz : 1);
        for (int32_t e = 0; e < nnz; ++e) s->cptr[p->colidx[e] + 1]++;
        for (int32_t j = 0; j < n; ++j) s->cptr[j + 1] += s->cptr[j];
        int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
        memcpy(fill, s->cptr, sizeof(int32_t) * ((size_t)n + 1));
        for (int32_t i = 0; i < m; ++i)
            for (int32_t e = p->rowptr[i]; e < p->rowptr[i + 1]; ++e) {
                const int32_t k = fill[p->colidx[e]]++;
                s->crow[k] = i;
                s->cval[k] = s->val[e];
            }
        free(fill);
    }
    s->c = dalloc(n); s->lv = dalloc(n); s->uv = dalloc(n);
    s->lc = dalloc(m); s->uc = dalloc(m);
    set_vectors(s);
    /* Q~ = D_c Q D_c */
    if (p->q_kind == 1) {
        size_t qn = (size_t)p->q_rowptr[n];
        s->qval = dalloc(qn);
        for (int32_t k = 0; k < n; ++k)
            for (int32_t e = p->q_rowptr[k]; e < p->q_rowptr[k + 1]; ++e)
                s->qval[e] = (s->dc[k] * p->q_val[e]) * s->dc[p->q_colidx[e]];
    } else if (p->q_kind == 2) {
        const int32_t r = p->q_rank;
        s->qf = dalloc((size_t)n * r);
        s->qd = dalloc(n);
        for (int32_t j = 0; j < n; ++j) {
            for (int32_t q = 0; q < r; ++q)
                s->qf[(size_t)j * r + q] = s->dc[j] * p->q_factor[(size_t)j * r + q];
            s->qd[j] = (s->dc[j] * s->dc[j]) * p->q_diag[j];
        }
    }
    /* step size: eta = safety / ||A~||_2 (1 when A~ = 0) */
    s->norm_a = power_norm_a(s, &s->power_iters);
    s->eta = s->norm_a > 0.0 ? s->o.step_safety / s->norm_a : 1.0;
    s->norm_q = power_norm_q(s);
    return s;
}

/* Threads of the products (OpenMP); 0 when built without OpenMP. */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 0;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

void orc_destroy(orc_ctx *s) {
    if (!s) return;
    free(s->val); free(s->qval); free(s->qf); free(s->qd);
    free(s->cptr); free(s->crow); free(s->cval);
    free(s->dr); free(s->dc); free(s->c); free(s->lc); free(s->uc);
    free(s->lv); free(s->uv);
    free(s);
}

void orc_scaling(const orc_ctx *s, double *dr, double *dc, double *eta, double *omega,
                 double *norm_a, double *norm_q, int32_t *power_iters) {
    if (dr) memcpy(dr, s->dr, sizeof(double) * s->m);
    if (dc) memcpy(dc, s->dc, sizeof(double) * s->n);
    if (eta) *eta = s->eta;
    if (omega) *omega = s->omega0;
    if (norm_a) *norm_a = s->norm_a;
    if (norm_q) *norm_q = s->norm_q;
    if (power_iters) *power_iters = s->power_iters;
}

void orc_pin_steps(orc_ctx *s, double eta, double norm_q) {
    s->eta = eta;
    s->norm_q = norm_q;
}

void orc_scaled_vectors(const orc_ctx *s, double *c, double *lc, double *uc, double *lv,
                        double *uv) {
    if (c) memcpy(c, s->c, sizeof(double) * s->n);
    if (lv) memcpy(lv, s->lv, sizeof(double) * s->n);
    if (uv) memcpy(uv, s->uv, sizeof(double) * s->n);
    if (lc) memcpy(lc, s->lc, sizeof(double) * s->m);
    if (uc) memcpy(uc, s->uc, sizeof(double) * s->m);
}

/* ------------------------------------------------------------------------ */
/* one iteration                                                             */

/* Dual proximal step of eq. (pdhg-lp): with v = y/sigma - a,
 * yhat = y - sigma a - sigma proj_[-u_c, -l_c](v) = sigma (v - proj(v)). */
static double dual_prox(double y, double a, double sigma, double lc, double uc) {
    double v = y / sigma - a;
    double pr = clampd(v, -uc, -lc);
    return sigma * (v - pr);
}

void orc_lp_step(const orc_ctx *s, const double *x, const double *y, const double *x0,
                 const double *y0, int64_t k, double tau, double sigma, double gamma,
                 double *xhat, double *yhat, double *xnew, double *ynew) {
    const int32_t m = s->m, n = s->n;
    double *aty = dalloc(n), *xh = dalloc(n), *xe = dalloc(n), *a = dalloc(m),
           *yh = dalloc(m);
    /* primal step: xhat = proj_X(x - tau (c - A'y)) */
    at_mul(s, y, aty);
    for (int32_t j = 0; j < n; ++j) {
        xh[j] = clampd(x[j] - tau * (s->c[j] - aty[j]), s->lv[j], s->uv[j]);
        xe[j] = 2.0 * xh[j] - x[j];
    }
    /* dual step with the extrapolated primal point 2 xhat - x */
    a_mul(s, xe, a);
    for (int32_t i = 0; i < m; ++i) yh[i] = dual_prox(y[i], a[i], sigma, s->lc[i], s->uc[i]);
    /* Halpern step with reflection, eq. (hrpdhg) */
    const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
    if (xnew)
        for (int32_t j = 0; j < n; ++j)
            xnew[j] = ak * ((1.0 + gamma) * xh[j] - gamma * x[j]) + bk * x0[j];
    if (ynew)
        for (int32_t i = 0; i < m; ++i)
            ynew[i] = ak * ((1.0 + gamma) * yh[i] - gamma * y[i]) + bk * y0[i];
    if (xhat) memcpy(xhat, xh, sizeof(double) * n);
    if (yhat) memcpy(yhat, yh, sizeof(double) * m);
    free(aty); free(xh); free(xe); free(a); free(yh);
}

/* rAPDHG step, Algorithm 2: beta_k = theta_k = 2/(k+2),
 * 1/tau_k = omega/eta + 2 ||Q~|| / (k+1), sigma = eta omega. */
void orc_qp_step(const orc_ctx *s, const double *x, const double *y, const double *xbar,
                 const double *ybar, int64_t k, double omega, double *xn, double *yn,
                 double *xbarn, double *ybarn) {
    const int32_t m = s->m, n = s->n;
    const double beta = 2.0 / (double)(k + 2), theta = beta;
    const double tau = 1.0 / (omega / s->eta + 2.0 * s->norm_q / (double)(k + 1));
    const double sigma = s->eta * omega;
    double *v = dalloc(n), *qv = dalloc(n), *aty = dalloc(n), *xh = dalloc(n),
           *xe = dalloc(n), *a = dalloc(m), *yh = dalloc(m);
    for (int32_t j = 0; j < n; ++j) v[j] = (1.0 - beta) * xbar[j] + beta * x[j];
    q_mul(s, v, qv);
    at_mul(s, y, aty);
    for (int32_t j = 0; j < n; ++j) {
        xh[j] = clampd(x[j] - tau * (qv[j] + s->c[j] - aty[j]), s->lv[j], s->uv[j]);
        xe[j] = 2.0 * xh[j] - x[j];
    }
    a_mul(s, xe, a);
    for (int32_t i = 0; i < m; ++i) yh[i] = dual_prox(y[i], a[i], sigma, s->lc[i], s->uc[i]);
    if (xbarn)
        for (int32_t j = 0; j < n; ++j) xbarn[j] = (1.0 - theta) * xbar[j] + theta * xh[j];
    if (ybarn)
        for (int32_t i = 0; i < m; ++i) ybarn[i] = (1.0 - theta) * ybar[i] + theta * yh[i];
    if (xn) memcpy(xn, xh, sizeof(double) * n);
    if (yn) memcpy(yn, yh, sizeof(double) * m);
    free(v); free(qv); free(aty); free(xh); free(xe); free(a); free(yh);
}

/* ||z - zhat||_M with M = [[I/tau, A~'], [A~, I/sigma]], the norm in which
 * the PDHG operator is firmly non-expansive:
 * r^2 = ||dx||^2/tau + ||dy||^2/sigma + 2 dy' A~ dx. */
double orc_fixed_point_residual(const orc_ctx *s, const double *x, const double *y,
                                const double *xhat, const double *yhat, double tau,
                                double sigma) {
    const int32_t m = s->m, n = s->n;
    double *dx = dalloc(n), *dy = dalloc(m), *adx = dalloc(m);
    for (int32_t j = 0; j < n; ++j) dx[j] = xhat[j] - x[j];
    for (int32_t i = 0; i < m; ++i) dy[i] = yhat[i] - y[i];
    a_mul(s, dx, adx);
    ld r2 = sumsq(dx, n) / tau + sumsq(dy, m) / sigma + 2.0L * dot(dy, adx, m);
    free(dx); free(dy); free(adx);
    return r2 > 0.0L ? (double)sqrtl(r2) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* relative KKT error, original space                                        */

void orc_kkt(const orc_problem *p, const double *x, const double *y, orc_result *r) {
    const int32_t m = p->m, n = p->n;
    double *ax = dalloc(m), *aty = dalloc(n), *qx = dalloc(n);
    /* A x and A' y with the original matrix */
    for (int32_t i = 0; i < m; ++i) {
        ld acc = 0.0L;
        if (p->dense) {
            for (int32_t j = 0; j < n; ++j) acc += (ld)p->dense[(size_t)i * n + j] * (ld)x[j];
        } else {
            for (int32_t e = p->rowptr[i]; e < p->rowptr[i + 1]; ++e)
                acc += (ld)p->val[e] * (ld)x[p->colidx[e]];
        }
        ax[i] = (double)acc;
    }
    {
        ld *acc = lalloc(n);
        for (int32_t i = 0; i < m; ++i) {
            if (p->dense) {
                for (int32_t j = 0; j < n; ++j) acc[j] += (ld)p->dense[(size_t)i * n + j] * (ld)y[i];
            } else {
                for (int32_t e = p->rowptr[i]; e < p->rowptr[i + 1]; ++e)
                    acc[p->colidx[e]] += (ld)p->val[e] * (ld)y[i];
            }
        }
        for (int32_t j = 0; j < n; ++j) aty[j] = (double)acc[j];
        free(acc);
    }
    q_mul_orig(p, x, qx);
    ld rp2 = 0.0L, rd2 = 0.0L, b2 = 0.0L, c2 = 0.0L;
    ld xqx = 0.0L, cx = 0.0L, dual_b = 0.0L, dual_v = 0.0L;
    for (int32_t i = 0; i < m; ++i) {
        /* primal residual: distance of A x to [l_c, u_c] */
        double rp = ax[i] - clampd(ax[i], p->lc[i], p->uc[i]);
        rp2 += (ld)rp * rp;
        double b = 0.0;
        if (isfinite(p->lc[i])) b = fmax(b, fabs(p->lc[i]));
        if (isfinite(p->uc[i])) b = fmax(b, fabs(p->uc[i]));
        b2 += (ld)b * b;
        /* -p(y) = l_c' y^+ - u_c' y^- (terms with infinite bounds are 0) */
        if (isfinite(p->lc[i])) dual_b += (ld)p->lc[i] * (ld)fmax(y[i], 0.0);
        if (isfinite(p->uc[i])) dual_b -= (ld)p->uc[i] * (ld)fmax(-y[i], 0.0);
    }
    for (int32_t j = 0; j < n; ++j) {
        /* gradient of the Lagrangian in x, and its part in the normal cone of X */
        double g = qx[j] + p->c[j] - aty[j];
        int lf = isfinite(p->lv[j]), uf = isfinite(p->uv[j]);
        double lam;
        if (!lf && !uf) lam = 0.0;
        else if (lf && !uf) lam = fmax(g, 0.0);
        else if (!lf && uf) lam = fmin(g, 0.0);
        else lam = g;
        double rd = g - lam;
        rd2 += (ld)rd * rd;
        c2 += (ld)p->c[j] * p->c[j];
        xqx += (ld)x[j] * (ld)qx[j];
        cx += (ld)p->c[j] * (ld)x[j];
        if (lf) dual_v += (ld)p->lv[j] * (ld)fmax(lam, 0.0);
        if (uf) dual_v -= (ld)p->uv[j] * (ld)fmax(-lam, 0.0);
    }
    ld P = 0.5L * xqx + cx;
    ld D = -0.5L * xqx + dual_b + dual_v;
    r->primal_obj = (double)P;
    r->dual_obj = (double)D;
    r->abs_primal = (double)sqrtl(rp2);
    r->abs_dual = (double)sqrtl(rd2);
    r->abs_gap = (double)fabsl(P - D);
    r->rel_primal = (double)(sqrtl(rp2) / (1.0L + sqrtl(b2)));
    r->rel_dual = (double)(sqrtl(rd2) / (1.0L + sqrtl(c2)));
    r->rel_gap = (double)(fabsl(P - D) / (1.0L + fabsl(P) + fabsl(D)));
    double k = r->rel_primal;
    if (r->rel_dual > k || isnan(r->rel_dual)) k = r->rel_dual;
    if (r->rel_gap > k || isnan(r->rel_gap)) k = r->rel_gap;
    r->kkt = k;
    free(ax); free(aty); free(qx);
}

/* ------------------------------------------------------------------------ */
/* solver loops                                                              */

static void unscale(const orc_ctx *s, const double *xs, const double *ys, double *x,
                    double *y) {
    for (int32_t j = 0; j < s->n; ++j) x[j] = s->dc[j] * xs[j];
    for (int32_t i = 0; i < s->m; ++i) y[i] = s->dr[i] * ys[i];
}

/* projection onto Y (sign constraints of the dual, Section 2) */
static double proj_y(double y, double lc, double uc) {
    double lo = isfinite(uc) ? -INFINITY : 0.0;   /* no upper bound: y >= 0 */
    double hi = isfinite(lc) ? INFINITY : 0.0;    /* no lower bound: y <= 0 */
    return clampd(y, lo, hi);
}

static void init_point(const orc_ctx *s, const double *x_init, const double *y_init,
                       double *x, double *y) {
    for (int32_t j = 0; j < s->n; ++j)
        x[j] = clampd(x_init ? x_init[j] / s->dc[j] : 0.0, s->lv[j], s->uv[j]);
    for (int32_t i = 0; i < s->m; ++i)
        y[i] = proj_y(y_init ? y_init[i] / s->dr[i] : 0.0, s->lc[i], s->uc[i]);
}

/* Infeasibility certificates (Section 3 lists infeasibility detection among
 * the solver's heuristics and Appendix A gives its tolerances; the tests are
 * the usual Farkas-type ray tests). The candidate rays are the differences
 * between the PDHG point and the restart anchor, in the original space:
 * dx = D_c (xh - x0), dy = D_r (yh - y0).
 *  - dual ray: yp = proj_Y(dy), g = -A'dy, lam = the part of g in the cone of
 *    the variable bounds; its objective l_c'yp+ - u_c'yp- + l_v'lam+ - u_v'lam-
 *    must be positive and the largest violation |dy - yp|, |g - lam| at most
 *    eps_primal_infeasible times it: the LP has no feasible point;
 *  - primal ray: c'dx < 0 and the largest violation of A dx in the recession
 *    cone of [l_c, u_c], of dx in that of [l_v, u_v] and, for a QP, of
 *    Q dx = 0 (the objective is linear along dx) at most
 *    eps_dual_infeasible |c'dx|: the objective is unbounded below.
 * Returns 2 or 3 and writes the ray scaled to objective 1 (dual) or -1
 * (primal) to ray_y / ray_x; 0 when neither test holds. */
static int infeasibility(const orc_ctx *s, const double *xh, const double *yh, const double *x0,
                         const double *y0, double *ray_x, double *ray_y) {
    const orc_problem *p = &s->p;
    const int32_t m = s->m, n = s->n;
    double *dx = dalloc(n), *dy = dalloc(m), *a = dalloc(m);
    ld *aty = lalloc(n);
    for (int32_t j = 0; j < n; ++j) dx[j] = s->dc[j] * (xh[j] - x0[j]);
    for (int32_t i = 0; i < m; ++i) dy[i] = s->dr[i] * (yh[i] - y0[i]);
    for (int32_t i = 0; i < m; ++i) {
        ld acc = 0.0L;
        if (p->dense) {
            for (int32_t j = 0; j < n; ++j) {
                acc += (ld)p->dense[(size_t)i * n + j] * (ld)dx[j];
                aty[j] += (ld)p->dense[(size_t)i * n + j] * (ld)dy[i];
            }
        } else {
            for (int32_t e = p->rowptr[i]; e < p->rowptr[i + 1]; ++e) {
                acc += (ld)p->val[e] * (ld)dx[p->colidx[e]];
                aty[p->colidx[e]] += (ld)p->val[e] * (ld)dy[i];
            }
        }
        a[i] = (double)acc;
    }
    int found = 0;
    /* dual ray */
    ld obj_d = 0.0L;
    double viol_d = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        const double yp = proj_y(dy[i], p->lc[i], p->uc[i]);
        viol_d = fmax(viol_d, fabs(dy[i] - yp));
        if (isfinite(p->lc[i])) obj_d += (ld)p->lc[i] * (ld)fmax(yp, 0.0);
        if (isfinite(p->uc[i])) obj_d -= (ld)p->uc[i] * (ld)fmax(-yp, 0.0);
    }
    for (int32_t j = 0; j < n; ++j) {
        const double g = -(double)aty[j];
        const int lf = isfinite(p->lv[j]), uf = isfinite(p->uv[j]);
        double lam;
        if (!lf && !uf) lam = 0.0;
        else if (lf && !uf) lam = fmax(g, 0.0);
        else if (!lf && uf) lam = fmin(g, 0.0);
        else lam = g;
        viol_d = fmax(viol_d, fabs(g - lam));
        if (lf) obj_d += (ld)p->lv[j] * (ld)fmax(lam, 0.0);
        if (uf) obj_d -= (ld)p->uv[j] * (ld)fmax(-lam, 0.0);
    }
    if (s->o.eps_primal_infeasible > 0.0 && obj_d > 0.0L &&
        viol_d <= s->o.eps_primal_infeasible * (double)obj_d) {
        for (int32_t i = 0; i < m; ++i) ray_y[i] = dy[i] / (double)obj_d;
        found = 2;
    }
    /* primal ray */
    if (!found) {
        ld obj_p = 0.0L;
        double viol_p = 0.0;
        for (int32_t j = 0; j < n; ++j) {
            obj_p += (ld)p->c[j] * (ld)dx[j];
            const double lo = isfinite(p->lv[j]) ? 0.0 : -INFINITY;
            const double hi = isfinite(p->uv[j]) ? 0.0 : INFINITY;
            viol_p = fmax(viol_p, fabs(dx[j] - clampd(dx[j], lo, hi)));
        }
        for (int32_t i = 0; i < m; ++i) {
            const double lo = isfinite(p->lc[i]) ? 0.0 : -INFINITY;
            const double hi = isfinite(p->uc[i]) ? 0.0 : INFINITY;
            viol_p = fmax(viol_p, fabs(a[i] - clampd(a[i], lo, hi)));
        }
        if (p->q_kind != 0) {
            double *qdx = dalloc(n);
            q_mul_orig(p, dx, qdx);
            for (int32_t j = 0; j < n; ++j) viol_p = fmax(viol_p, fabs(qdx[j]));
            free(qdx);
        }
        if (s->o.eps_dual_infeasible > 0.0 && obj_p < 0.0L &&
            viol_p <= s->o.eps_dual_infeasible * (double)(-obj_p)) {
            for (int32_t j = 0; j < n; ++j) ray_x[j] = dx[j] / (double)(-obj_p);
            found = 3;
        }
    }
    free(dx); free(dy); free(a); free(aty);
    return found;
}

/* Restart test shared by both methods: sufficient decay, necessary decay
 * without local progress, or an artificial restart after a long cycle. */
static int restart_due(const orc_ctx *s, double r, double r_start, double r_prev,
                       int64_t k, int64_t t) {
    if (r <= s->o.restart_sufficient * r_start) return 1;
    if (r <= s->o.restart_necessary * r_start && r > r_prev) return 1;
    if ((double)k >= s->o.restart_artificial * (double)t) return 1;
    return 0;
}

/* primal weight after a restart: log-smoothing (weight 1/2) towards dy/dx */
static double new_weight(double omega, double dxr, double dyr) {
    if (dxr > 1e-10 && dyr > 1e-10) return exp(0.5 * log(dyr / dxr) + 0.5 * log(omega));
    return omega;
}

/* Core LP loop (Algorithm 1). When frozen != NULL the loop runs exactly T
 * iterations and takes restarts / weights from the schedule instead of the
 * tests; rec_* record the schedule actually used; masks (optional) record
 * the projection state of every iteration for the reverse pass. */
typedef struct {
    const uint8_t *restart;   /* [T] or NULL */
    const double *omega;      /* [T] or NULL */
    uint8_t *rec_restart;     /* [T] or NULL */
    double *rec_omega;        /* [T] or NULL */
    uint8_t *xmask;           /* [T*n]: 1 if xhat strictly inside its box */
    uint8_t *ymask;           /* [T*m]: 0 interior, 1 at -u_c, 2 at -l_c */
    int64_t *kk;              /* [T]: inner counter */
    int64_t T;
} lp_trace;

static int lp_loop(orc_ctx *s, const double *x_init, const double *y_init, double *x_out,
                   double *y_out, orc_result *res, lp_trace *tr) {
    const int32_t m = s->m, n = s->n;
    double *x = dalloc(n), *y = dalloc(m), *x0 = dalloc(n), *y0 = dalloc(m);
    double *xh = dalloc(n), *yh = dalloc(m), *xn = dalloc(n), *yn = dalloc(m);
    double *xo = dalloc(n), *yo = dalloc(m);
    double *ray_x = dalloc(n), *ray_y = dalloc(m);
    init_point(s, x_init, y_init, x, y);
    memcpy(x0, x, sizeof(double) * n);
    memcpy(y0, y, sizeof(double) * m);
    double omega = s->omega0, tau = s->eta / omega, sigma = s->eta * omega;
    double r_start = 0.0, r_prev = 0.0;
    int64_t k = 0, t = 0, nr = 0;
    const int64_t limit = tr ? tr->T : s->o.iteration_limit;
    int status = 0;
    memset(res, 0, sizeof(*res));
    for (;;) {
        if (tr && tr->omega) {
            omega = tr->omega[t];
            tau = s->eta / omega;
            sigma = s->eta * omega;
        }
        if (tr && tr->rec_omega) tr->rec_omega[t] = omega;
        orc_lp_step(s, x, y, x0, y0, k, tau, sigma, s->o.gamma, xh, yh, xn, yn);
        if (tr && tr->xmask) {
            /* record the projection state for the reverse pass */
            double *aty = dalloc(n), *xe = dalloc(n), *a = dalloc(m);
            at_mul(s, y, aty);
            for (int32_t j = 0; j < n; ++j) {
                double u = x[j] - tau * (s->c[j] - aty[j]);
                tr->xmask[t * n + j] = (u > s->lv[j] && u < s->uv[j]) ? 1 : 0;
                xe[j] = 2.0 * xh[j] - x[j];
            }
            a_mul(s, xe, a);
            for (int32_t i = 0; i < m; ++i) {
                double v = y[i] / sigma - a[i];
                tr->ymask[t * m + i] = v < -s->uc[i] ? 1 : (v > -s->lc[i] ? 2 : 0);
            }
            tr->kk[t] = k;
            free(aty); free(xe); free(a);
        }
        const int is_check = (t % s->o.check_every) == 0;
        const int is_last = (t + 1 >= limit);
        if (!tr && (is_check || is_last)) {
            unscale(s, xh, yh, xo, yo);
            orc_kkt(&s->p, xo, yo, res);
            if (s->o.verbose)
                fprintf(stderr, "oracle t=%lld k=%lld nr=%lld omega=%.3e kkt=%.3e (%.2e %.2e %.2e)\n",
                        (long long)t, (long long)k, (long long)nr, omega, res->kkt,
                        res->rel_primal, res->rel_dual, res->rel_gap);
            if (isnan(res->kkt)) { status = 6; break; }
            /* a polishing phase stops on its own residual alone */
            const double tv = s->polish == 1 ? res->rel_primal : s->polish == 2 ? res->rel_dual : res->kkt;
            if (tv <= (s->polish ? s->o.eps_feas_polish : s->o.eps)) { status = 1; break; }
            /* rays from the anchor are tested once a restart has set it */
            if (nr > 0 && !s->polish) {
                status = infeasibility(s, xh, yh, x0, y0, ray_x, ray_y);
                if (status) break;
            }
        }
        if (is_last) { status = 4; break; }
        int restart = 0;
        double r = 0.0;
        if (tr && tr->restart) {
            restart = tr->restart[t];
        } else if (is_check) {
            r = orc_fixed_point_residual(s, x, y, xh, yh, tau, sigma);
            if (s->o.verbose)
                fprintf(stderr, "oracle   r=%.17e r/r_start=%.17e r_prev=%.17e\n", r,
                        r_start > 0 ? r / r_start : 0.0, r_prev);
            if (t == 0) { r_start = r; r_prev = r; }
            else if (restart_due(s, r, r_start, r_prev, k, t)) restart = 1;
            else r_prev = r;
        }
        if (tr && tr->rec_restart) tr->rec_restart[t] = (uint8_t)restart;
        if (restart) {
            ld dx2 = 0.0L, dy2 = 0.0L;
            for (int32_t j = 0; j < n; ++j) dx2 += (ld)(xh[j] - x0[j]) * (xh[j] - x0[j]);
            for (int32_t i = 0; i < m; ++i) dy2 += (ld)(yh[i] - y0[i]) * (yh[i] - y0[i]);
            memcpy(x, xh, sizeof(double) * n); memcpy(x0, xh, sizeof(double) * n);
            memcpy(y, yh, sizeof(double) * m); memcpy(y0, yh, sizeof(double) * m);
            if (!(tr && tr->omega)) {
                omega = new_weight(omega, (double)sqrtl(dx2), (double)sqrtl(dy2));
                tau = s->eta / omega;
                sigma = s->eta * omega;
            }
            k = 0;
            r_start = r;
            r_prev = r;
            ++nr;
        } else {
            memcpy(x, xn, sizeof(double) * n);
            memcpy(y, yn, sizeof(double) * m);
            ++k;
        }
        ++t;
    }
    unscale(s, xh, yh, x_out, y_out);
    if (status == 2) memcpy(y_out, ray_y, sizeof(double) * m);
    if (status == 3) memcpy(x_out, ray_x, sizeof(double) * n);
    if (tr) orc_kkt(&s->p, x_out, y_out, res);
    res->status = status;
    res->iterations = t + 1;
    res->restarts = nr;
    res->eta = s->eta;
    res->omega = omega;
    res->norm_a = s->norm_a;
    res->norm_q = s->norm_q;
    res->power_iters = s->power_iters;
    free(x); free(y); free(x0); free(y0); free(xh); free(yh); free(xn); free(yn);
    free(xo); free(yo); free(ray_x); free(ray_y);
    return status;
}

/* rAPDHG loop (Algorithm 2); the check uses the weighted KKT norm
 * sqrt(omega ||r_p||^2 + ||r_d||^2 / omega + gap^2) as restart metric. */
static int qp_loop(orc_ctx *s, const double *x_init, const double *y_init, double *x_out,
                   double *y_out, orc_result *res) {
    const int32_t m = s->m, n = s->n;
    double *x = dalloc(n), *y = dalloc(m), *xb = dalloc(n), *yb = dalloc(m);
    double *x0 = dalloc(n), *y0 = dalloc(m);
    double *xn = dalloc(n), *yn = dalloc(m), *xbn = dalloc(n), *ybn = dalloc(m);
    double *xo = dalloc(n), *yo = dalloc(m);
    double *ray_x = dalloc(n), *ray_y = dalloc(m);
    init_point(s, x_init, y_init, x, y);
    memcpy(xb, x, sizeof(double) * n); memcpy(yb, y, sizeof(double) * m);
    memcpy(x0, x, sizeof(double) * n); memcpy(y0, y, sizeof(double) * m);
    double omega = s->omega0;
    double r_start = 0.0, r_prev = 0.0;
    int64_t k = 0, t = 0, nr = 0;
    int status = 0;
    memset(res, 0, sizeof(*res));
    for (;;) {
        orc_qp_step(s, x, y, xb, yb, k, omega, xn, yn, xbn, ybn);
        memcpy(x, xn, sizeof(double) * n); memcpy(y, yn, sizeof(double) * m);
        memcpy(xb, xbn, sizeof(double) * n); memcpy(yb, ybn, sizeof(double) * m);
        const int is_check = (t % s->o.check_every) == 0;
        const int is_last = (t + 1 >= s->o.iteration_limit);
        double r = 0.0;
        if (is_check || is_last) {
            unscale(s, xb, yb, xo, yo);
            orc_kkt(&s->p, xo, yo, res);
            if (s->o.verbose)
                fprintf(stderr, "oracle-qp t=%lld k=%lld nr=%lld omega=%.3e kkt=%.3e\n",
                        (long long)t, (long long)k, (long long)nr, omega, res->kkt);
            if (isnan(res->kkt)) { status = 6; break; }
            if (res->kkt <= s->o.eps) { status = 1; break; }
            /* rays from the anchor (averages minus restart point), as for LPs */
            if (nr > 0) {
                status = infeasibility(s, xb, yb, x0, y0, ray_x, ray_y);
                if (status) break;
            }
            r = sqrt(omega * res->abs_primal * res->abs_primal +
                     res->abs_dual * res->abs_dual / omega + res->abs_gap * res->abs_gap);
        }
        if (is_last) { status = 4; break; }
        int restart = 0;
        if (is_check) {
            if (t == 0) { r_start = r; r_prev = r; }
            else if (restart_due(s, r, r_start, r_prev, k, t)) restart = 1;
            else r_prev = r;
        }
        if (restart) {
            ld dx2 = 0.0L, dy2 = 0.0L;
            for (int32_t j = 0; j < n; ++j) dx2 += (ld)(xb[j] - x0[j]) * (xb[j] - x0[j]);
            for (int32_t i = 0; i < m; ++i) dy2 += (ld)(yb[i] - y0[i]) * (yb[i] - y0[i]);
            memcpy(x, xb, sizeof(double) * n); memcpy(x0, xb, sizeof(double) * n);
            memcpy(y, yb, sizeof(double) * m); memcpy(y0, yb, sizeof(double) * m);
            omega = new_weight(omega, (double)sqrtl(dx2), (double)sqrtl(dy2));
            k = 0;
            r_start = r;
            r_prev = r;
            ++nr;
        } else {
            ++k;
        }
        ++t;
    }
    unscale(s, xb, yb, x_out, y_out);
    if (status == 2) memcpy(y_out, ray_y, sizeof(double) * m);
    if (status == 3) memcpy(x_out, ray_x, sizeof(double) * n);
    res->status = status;
    res->iterations = t + 1;
    res->restarts = nr;
    res->eta = s->eta;
    res->omega = omega;
    res->norm_a = s->norm_a;
    res->norm_q = s->norm_q;
    res->power_iters = s->power_iters;
    free(x); free(y); free(xb); free(yb); free(x0); free(y0); free(ray_x); free(ray_y);
    free(xn); free(yn); free(xbn); free(ybn); free(xo); free(yo);
    return status;
}

/* Feasibility polishing (Section 3: a post-processing step that solves the
 * feasibility-only problem from the current point, to eps_feas_polish,
 * Appendix A). Reading: two phases on the same scaled matrix,
 *  - primal: the LP with c = 0 from (x, 0) until the relative primal
 *    residual is <= eps_feas_polish;
 *  - dual: the LP with every finite bound set to 0 (the problem whose dual
 *    constraints are those of the LP and whose objective is 0) from (0, y)
 *    until the relative dual residual is <= eps_feas_polish;
 * the polished point is (x of the primal phase, y of the dual phase). Both
 * residuals depend only on A, c and which bounds are finite, so they hold
 * for the original LP too; its gap is reported as measured. x, y: original
 * space, in and out; res gets the KKT terms of the polished point. */
static void polish(orc_ctx *s, double *x, double *y, orc_result *res) {
    const int32_t m = s->m, n = s->n;
    const orc_problem saved = s->p;
    double *zc = dalloc(n), *lc = dalloc(m), *uc = dalloc(m), *lv = dalloc(n), *uv = dalloc(n);
    double *xp = dalloc(n), *yp = dalloc(m), *xd = dalloc(n), *yd = dalloc(m);
    for (int32_t i = 0; i < m; ++i) {
        lc[i] = isfinite(saved.lc[i]) ? 0.0 : saved.lc[i];
        uc[i] = isfinite(saved.uc[i]) ? 0.0 : saved.uc[i];
    }
    for (int32_t j = 0; j < n; ++j) {
        lv[j] = isfinite(saved.lv[j]) ? 0.0 : saved.lv[j];
        uv[j] = isfinite(saved.uv[j]) ? 0.0 : saved.uv[j];
    }
    orc_result r1, r2;
    s->p.c = zc;
    set_vectors(s);
    s->polish = 1;
    lp_loop(s, x, NULL, xp, yp, &r1, NULL);
    s->p = saved;
    s->p.lc = lc; s->p.uc = uc; s->p.lv = lv; s->p.uv = uv;
    set_vectors(s);
    s->polish = 2;
    lp_loop(s, NULL, y, xd, yd, &r2, NULL);
    s->p = saved;
    set_vectors(s);
    s->polish = 0;
    memcpy(x, xp, sizeof(double) * n);
    memcpy(y, yd, sizeof(double) * m);
    const orc_result before = *res;
    orc_kkt(&s->p, x, y, res);
    res->status = before.status;
    res->iterations = before.iterations + r1.iterations + r2.iterations;
    res->restarts = before.restarts;
    res->eta = before.eta;
    res->omega = before.omega;
    res->norm_a = before.norm_a;
    res->norm_q = before.norm_q;
    res->power_iters = before.power_iters;
    res->polish_iterations = r1.iterations + r2.iterations;
    free(zc); free(lc); free(uc); free(lv); free(uv); free(xp); free(yp); free(xd); free(yd);
}

int orc_solve(orc_ctx *s, const double *x_init, const double *y_init, double *x_out,
              double *y_out, orc_result *res) {
    if (s->p.q_kind != 0) return qp_loop(s, x_init, y_init, x_out, y_out, res);
    int st = lp_loop(s, x_init, y_init, x_out, y_out, res, NULL);
    if (st == 1 && s->o.feasibility_polishing) polish(s, x_out, y_out, res);
    return st;
}

/* ------------------------------------------------------------------------ */
/* unrolled LP and its reverse pass (frozen schedule)                         */

int orc_unrolled_lp(orc_ctx *s, int64_t T, const uint8_t *sched_restart,
                    const double *sched_omega, uint8_t *rec_restart, double *rec_omega,
                    double *x_out, double *y_out) {
    if (T < 1 || s->p.q_kind != 0) return -1;
    lp_trace tr;
    memset(&tr, 0, sizeof(tr));
    tr.T = T;
    tr.restart = sched_restart;
    tr.omega = sched_omega;
    tr.rec_restart = rec_restart;
    tr.rec_omega = rec_omega;
    orc_result res;
    lp_loop(s, NULL, NULL, x_out, y_out, &res, &tr);
    return 0;
}

/* Reverse pass of T iterations (Algorithm 1 unrolled) given the schedule.
 * Per iteration, in reverse order of the forward equations:
 *   Halpern:   x' = a_k((1+g) xh - g x) + b_k x0 (same for y), anchors carried
 *   restart:   x' = x0' = xh, y' = y0' = yh
 *   dual:      yh = sigma (v - clamp(v, -u_c, -l_c)), v = y/sigma - A~ xe
 *   extrap.:   xe = 2 xh - x
 *   primal:    xh = clamp(u, l_v, u_v), u = x - tau (c - A~'y)
 * The projection states are recomputed by a forward replay. */
int orc_unrolled_lp_backward(orc_ctx *s, int64_t T, const uint8_t *sched_restart,
                             const double *sched_omega, const double *gx, const double *gy,
                             double *gc, double *glc, double *guc) {
    if (T < 1 || s->p.q_kind != 0 || !sched_restart || !sched_omega) return -1;
    const int32_t m = s->m, n = s->n;
    lp_trace tr;
    memset(&tr, 0, sizeof(tr));
    tr.T = T;
    tr.restart = sched_restart;
    tr.omega = sched_omega;
    tr.xmask = (uint8_t *)calloc((size_t)T * n, 1);
    tr.ymask = (uint8_t *)calloc((size_t)T * (m ? m : 1), 1);
    tr.kk = (int64_t *)calloc((size_t)T, sizeof(int64_t));
    double *xo = dalloc(n), *yo = dalloc(m);
    orc_result res;
    lp_loop(s, NULL, NULL, xo, yo, &res, &tr);
    /* cotangents of the state (x, y, x0, y0) after iteration t, and of the
     * PDHG point of the last iteration */
    double *bx = dalloc(n), *by = dalloc(m), *bx0 = dalloc(n), *by0 = dalloc(m);
    double *bxh = dalloc(n), *byh = dalloc(m), *bxe = dalloc(n), *ba = dalloc(m);
    double *bu = dalloc(n), *tmp_n = dalloc(n), *tmp_m = dalloc(m);
    ld *gcs = lalloc(n), *glcs = lalloc(m), *gucs = lalloc(m);
    const double g = s->o.gamma;
    for (int64_t t = T - 1; t >= 0; --t) {
        const double omega = sched_omega[t];
        const double tau = s->eta / omega, sigma = s->eta * omega;
        const int64_t k = tr.kk[t];
        memset(bxh, 0, sizeof(double) * n);
        memset(byh, 0, sizeof(double) * m);
        if (t == T - 1) {
            /* output is the unscaled PDHG point of the last iteration */
            for (int32_t j = 0; j < n; ++j) bxh[j] = s->dc[j] * gx[j];
            for (int32_t i = 0; i < m; ++i) byh[i] = s->dr[i] * gy[i];
        } else if (sched_restart[t]) {
            for (int32_t j = 0; j < n; ++j) { bxh[j] = bx[j] + bx0[j]; bx[j] = 0.0; bx0[j] = 0.0; }
            for (int32_t i = 0; i < m; ++i) { byh[i] = by[i] + by0[i]; by[i] = 0.0; by0[i] = 0.0; }
        } else {
            const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
            for (int32_t j = 0; j < n; ++j) {
                bxh[j] = ak * (1.0 + g) * bx[j];
                bx0[j] += bk * bx[j];
                bx[j] = -ak * g * bx[j];
            }
            for (int32_t i = 0; i < m; ++i) {
                byh[i] = ak * (1.0 + g) * by[i];
                by0[i] += bk * by[i];
                by[i] = -ak * g * by[i];
            }
        }
        if (t == T - 1) {
            memset(bx, 0, sizeof(double) * n); memset(by, 0, sizeof(double) * m);
            memset(bx0, 0, sizeof(double) * n); memset(by0, 0, sizeof(double) * m);
        }
        /* dual step */
        for (int32_t i = 0; i < m; ++i) {
            const uint8_t st = tr.ymask[t * m + i];
            double bv = 0.0;
            if (st == 0) bv = 0.0;                          /* yhat = 0 */
            else bv = sigma * byh[i];                        /* yhat = sigma (v + bound) */
            if (st == 1) gucs[i] += (ld)(sigma * byh[i]);
            if (st == 2) glcs[i] += (ld)(sigma * byh[i]);
            by[i] += bv / sigma;
            ba[i] = -bv;
        }
        at_mul(s, ba, bxe);
        for (int32_t j = 0; j < n; ++j) {
            bxh[j] += 2.0 * bxe[j];
            bx[j] -= bxe[j];
        }
        /* primal step */
        for (int32_t j = 0; j < n; ++j) {
            bu[j] = tr.xmask[t * n + j] ? bxh[j] : 0.0;
            bx[j] += bu[j];
            gcs[j] += (ld)(-tau * bu[j]);
            tmp_n[j] = tau * bu[j];
        }
        a_mul(s, tmp_n, tmp_m);
        for (int32_t i = 0; i < m; ++i) by[i] += tmp_m[i];
    }
    /* back to original data: c~ = D_c c, l~_c = D_r l_c, u~_c = D_r u_c */
    for (int32_t j = 0; j < n; ++j) gc[j] = s->dc[j] * (double)gcs[j];
    for (int32_t i = 0; i < m; ++i) {
        glc[i] = isfinite(s->p.lc[i]) ? s->dr[i] * (double)glcs[i] : 0.0;
        guc[i] = isfinite(s->p.uc[i]) ? s->dr[i] * (double)gucs[i] : 0.0;
    }
    free(tr.xmask); free(tr.ymask); free(tr.kk); free(xo); free(yo);
    free(bx); free(by); free(bx0); free(by0); free(bxh); free(byh); free(bxe); free(ba);
    free(bu); free(tmp_n); free(tmp_m); free(gcs); free(glcs); free(gucs);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* unrolled rAPDHG and its reverse pass (frozen schedule)                     */

/* Forward of T iterations; when `keep` is given, stores per iteration the
 * momentum point v, the box-interior mask of x and the clamp state of y, and
 * the inner counter. */
typedef struct {
    double *v;        /* [T*n] */
    uint8_t *xmask;   /* [T*n] */
    uint8_t *ymask;   /* [T*m] */
    int64_t *kk;      /* [T] */
} qp_trace;

static void qp_unrolled_core(orc_ctx *s, int64_t T, const uint8_t *sched_restart,
                             const double *sched_omega, uint8_t *rec_restart, double *rec_omega,
                             double *x_out, double *y_out, qp_trace *keep) {
    const int32_t m = s->m, n = s->n;
    double *x = dalloc(n), *y = dalloc(m), *xb = dalloc(n), *yb = dalloc(m);
    double *x0 = dalloc(n), *y0 = dalloc(m);
    double *v = dalloc(n), *qv = dalloc(n), *aty = dalloc(n), *xe = dalloc(n), *a = dalloc(m);
    double *xo = dalloc(n), *yo = dalloc(m);
    init_point(s, NULL, NULL, x, y);
    memcpy(xb, x, sizeof(double) * n); memcpy(yb, y, sizeof(double) * m);
    memcpy(x0, x, sizeof(double) * n); memcpy(y0, y, sizeof(double) * m);
    double omega = s->omega0, r_start = 0.0, r_prev = 0.0;
    int64_t k = 0;
    orc_result res;
    for (int64_t t = 0; t < T; ++t) {
        if (sched_omega) omega = sched_omega[t];
        if (rec_omega) rec_omega[t] = omega;
        const double beta = 2.0 / (double)(k + 2), theta = beta;
        const double tau = 1.0 / (omega / s->eta + 2.0 * s->norm_q / (double)(k + 1));
        const double sigma = s->eta * omega;
        for (int32_t j = 0; j < n; ++j) v[j] = (1.0 - beta) * xb[j] + beta * x[j];
        q_mul(s, v, qv);
        at_mul(s, y, aty);
        for (int32_t j = 0; j < n; ++j) {
            double u = x[j] - tau * (qv[j] + s->c[j] - aty[j]);
            double xp = clampd(u, s->lv[j], s->uv[j]);
            if (keep) {
                keep->v[t * n + j] = v[j];
                keep->xmask[t * n + j] = (u > s->lv[j] && u < s->uv[j]) ? 1 : 0;
            }
            xe[j] = 2.0 * xp - x[j];
            x[j] = xp;
            xb[j] = (1.0 - theta) * xb[j] + theta * xp;
        }
        a_mul(s, xe, a);
        for (int32_t i = 0; i < m; ++i) {
            double w = y[i] / sigma - a[i];
            if (keep) keep->ymask[t * m + i] = w < -s->uc[i] ? 1 : (w > -s->lc[i] ? 2 : 0);
            double yp = sigma * (w - clampd(w, -s->uc[i], -s->lc[i]));
            y[i] = yp;
            yb[i] = (1.0 - theta) * yb[i] + theta * yp;
        }
        if (keep) keep->kk[t] = k;
        if (t + 1 >= T) break;
        int restart = 0;
        if (sched_restart) {
            restart = sched_restart[t];
        } else if ((t % s->o.check_every) == 0) {
            unscale(s, xb, yb, xo, yo);
            orc_kkt(&s->p, xo, yo, &res);
            double r = sqrt(omega * res.abs_primal * res.abs_primal +
                            res.abs_dual * res.abs_dual / omega + res.abs_gap * res.abs_gap);
            if (t == 0) { r_start = r; r_prev = r; }
            else if (restart_due(s, r, r_start, r_prev, k, t)) restart = 1;
            else r_prev = r;
            if (restart) {
                ld dx2 = 0.0L, dy2 = 0.0L;
                for (int32_t j = 0; j < n; ++j) dx2 += (ld)(xb[j] - x0[j]) * (xb[j] - x0[j]);
                for (int32_t i = 0; i < m; ++i) dy2 += (ld)(yb[i] - y0[i]) * (yb[i] - y0[i]);
                omega = new_weight(omega, (double)sqrtl(dx2), (double)sqrtl(dy2));
                r_start = r;
                r_prev = r;
            }
        }
        if (rec_restart) rec_restart[t] = (uint8_t)restart;
        if (restart) {
            memcpy(x, xb, sizeof(double) * n); memcpy(x0, xb, sizeof(double) * n);
            memcpy(y, yb, sizeof(double) * m); memcpy(y0, yb, sizeof(double) * m);
            k = 0;
        } else {
            ++k;
        }
    }
    if (x_out) unscale(s, xb, yb, x_out, y_out);
    free(x); free(y); free(xb); free(yb); free(x0); free(y0); free(v); free(qv); free(aty);
    free(xe); free(a); free(xo); free(yo);
}

int orc_unrolled_qp(orc_ctx *s, int64_t T, const uint8_t *sched_restart, const double *sched_omega,
                    uint8_t *rec_restart, double *rec_omega, double *x_out, double *y_out) {
    if (T < 1 || s->p.q_kind == 0) return -1;
    qp_unrolled_core(s, T, sched_restart, sched_omega, rec_restart, rec_omega, x_out, y_out, NULL);
    return 0;
}

/* Reverse of Algorithm 2 per iteration (restarts and weights frozen):
 *   xbar+ = (1-th) xbar + th x+,  ybar+ likewise
 *   y+ = sigma (w - clamp(w, -u_c, -l_c)),  w = y/sigma - A~ xe,  xe = 2x+ - x
 *   x+ = clamp(u),  u = x - tau (Q~ v + c - A~'y),  v = (1-beta) xbar + beta x
 *   Q~ v = F~ (F~' v) + d~ v  (d~ = D_c^2 d) or a general symmetric Q~
 * A restart after iteration t makes the next iteration start from
 * (xbar+, ybar+, xbar+, ybar+). */
int orc_unrolled_qp_backward(orc_ctx *s, int64_t T, const uint8_t *sched_restart,
                             const double *sched_omega, const double *gx, const double *gy,
                             double *gc, double *glc, double *guc, double *gd) {
    if (T < 1 || s->p.q_kind == 0 || !sched_restart || !sched_omega) return -1;
    const int32_t m = s->m, n = s->n;
    qp_trace tr;
    tr.v = dalloc((size_t)T * n);
    tr.xmask = (uint8_t *)calloc((size_t)T * n, 1);
    tr.ymask = (uint8_t *)calloc((size_t)T * (m ? m : 1), 1);
    tr.kk = (int64_t *)calloc((size_t)T, sizeof(int64_t));
    qp_unrolled_core(s, T, sched_restart, sched_omega, NULL, NULL, NULL, NULL, &tr);
    double *bx = dalloc(n), *by = dalloc(m), *bxb = dalloc(n), *byb = dalloc(m);
    double *bxp = dalloc(n), *byp = dalloc(m), *bw = dalloc(m), *bxe = dalloc(n);
    double *bqv = dalloc(n), *bv = dalloc(n), *tmp = dalloc(n), *tm = dalloc(m);
    ld *gcs = lalloc(n), *gds = lalloc(n), *glcs = lalloc(m), *gucs = lalloc(m);
    /* cotangent of the output (unscaled averages after iteration T-1) */
    for (int32_t j = 0; j < n; ++j) bxb[j] = s->dc[j] * gx[j];
    for (int32_t i = 0; i < m; ++i) byb[i] = s->dr[i] * gy[i];
    for (int64_t t = T - 1; t >= 0; --t) {
        if (t < T - 1 && sched_restart[t]) {
            for (int32_t j = 0; j < n; ++j) { bxb[j] += bx[j]; bx[j] = 0.0; }
            for (int32_t i = 0; i < m; ++i) { byb[i] += by[i]; by[i] = 0.0; }
        }
        const int64_t k = tr.kk[t];
        const double omega = sched_omega[t];
        const double beta = 2.0 / (double)(k + 2), theta = beta;
        const double tau = 1.0 / (omega / s->eta + 2.0 * s->norm_q / (double)(k + 1));
        const double sigma = s->eta * omega;
        /* averages */
        for (int32_t j = 0; j < n; ++j) { bxp[j] = bx[j] + theta * bxb[j]; bxb[j] = (1.0 - theta) * bxb[j]; }
        for (int32_t i = 0; i < m; ++i) { byp[i] = by[i] + theta * byb[i]; byb[i] = (1.0 - theta) * byb[i]; }
        /* dual step */
        for (int32_t i = 0; i < m; ++i) {
            const uint8_t st = tr.ymask[t * m + i];
            bw[i] = st ? sigma * byp[i] : 0.0;
            if (st == 1) gucs[i] += (ld)(sigma * byp[i]);
            if (st == 2) glcs[i] += (ld)(sigma * byp[i]);
            by[i] = bw[i] / sigma;       /* w depends on the input y */
            tm[i] = -bw[i];
        }
        at_mul(s, tm, bxe);              /* d w / d xe = -A~ */
        for (int32_t j = 0; j < n; ++j) {
            bxp[j] += 2.0 * bxe[j];
            bx[j] = -bxe[j];
        }
        /* primal step */
        for (int32_t j = 0; j < n; ++j) {
            const double bu = tr.xmask[t * n + j] ? bxp[j] : 0.0;
            bx[j] += bu;
            bqv[j] = -tau * bu;
            gcs[j] += (ld)(-tau * bu);
            tmp[j] = tau * bu;
        }
        a_mul(s, tmp, tm);
        for (int32_t i = 0; i < m; ++i) by[i] += tm[i];
        /* Q~ v is symmetric: bv = Q~ bqv; d~ term */
        q_mul(s, bqv, bv);
        for (int32_t j = 0; j < n; ++j) {
            gds[j] += (ld)bqv[j] * (ld)tr.v[t * n + j];
            bxb[j] += (1.0 - beta) * bv[j];
            bx[j] += beta * bv[j];
        }
    }
    for (int32_t j = 0; j < n; ++j) {
        gc[j] = s->dc[j] * (double)gcs[j];
        if (gd) gd[j] = (s->p.q_kind == 2) ? (s->dc[j] * s->dc[j]) * (double)gds[j] : 0.0;
    }
    for (int32_t i = 0; i < m; ++i) {
        glc[i] = isfinite(s->p.lc[i]) ? s->dr[i] * (double)glcs[i] : 0.0;
        guc[i] = isfinite(s->p.uc[i]) ? s->dr[i] * (double)gucs[i] : 0.0;
    }
    free(tr.v); free(tr.xmask); free(tr.ymask); free(tr.kk);
    free(bx); free(by); free(bxb); free(byb); free(bxp); free(byp); free(bw); free(bxe);
    free(bqv); free(bv); free(tmp); free(tm); free(gcs); free(gds); free(glcs); free(gucs);
    return 0;
}
