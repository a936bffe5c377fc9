// rAPDHG for convex QPs (MPAX paper, Section 2.2, eq. (pdhg-momentum-qp) and
// Algorithm 2), scaled space, internal order.
//
// One iteration with inner counter k (beta = theta = 2/(k+2),
// 1/tau_k = omega/eta + 2 ||Q~||/(k+1), sigma = eta omega):
//   v = (1-beta) xbar + beta x;  qv = Q~ v            (Q operator kernels)
//   x+ = clamp(x - tau_k (qv + c - A~'y)), xext = 2x+ - x, xbar update   (primal)
//   y+ = dual prox with A~ xext, ybar update                             (dual)
// A check evaluates the KKT error of (xbar, ybar) in the original space and
// restarts on the weighted KKT norm sqrt(omega |r_p|^2 + |r_d|^2/omega + gap^2);
// a restart sets x, x0 <- xbar and y, y0 <- ybar.
#include "device.hpp"

namespace pdhg {

__device__ __forceinline__ int64_t qp_k(const DevState *st, int32_t j) {
    return j > 0 ? st->k_base + (j - 1) : (st->first ? 0 : st->k_base + st->plain_prev);
}

// v = (1-beta) xbar + beta x (mode 0) or v = xbar (mode 1); for a low-rank Q
// also the per-workgroup partial sums of F~'v (r values per workgroup).
__global__ __launch_bounds__(kBlock) void k_qp_v(const DevState *__restrict__ st, int32_t n,
                                                 int32_t j, int32_t mode, const double *__restrict__ x,
                                                 const double *__restrict__ xbar,
                                                 double *__restrict__ v,
                                                 const double *__restrict__ F, int32_t r,
                                                 double *__restrict__ partials) {
    if (st->done) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double vi = 0.0;
    if (i < n) {
        if (mode == 0) {
            const int64_t k = qp_k(st, j);
            const double beta = 2.0 / (double)(k + 2);
            vi = (1.0 - beta) * xbar[i] + beta * x[i];
        } else {
            vi = xbar[i];
        }
        v[i] = vi;
    }
    if (F) {
        for (int32_t q = 0; q < r; ++q) {
            double t[1] = {i < n ? F[(size_t)i * r + q] * vi : 0.0};
            block_sum_store<1>(t, partials + (size_t)blockIdx.x * r + q);
            __syncthreads();
        }
    }
}

// t_q = sum over workgroups of the partials, in workgroup order.
__global__ void k_qp_t(const DevState *__restrict__ st, const double *__restrict__ partials,
                       int32_t nb, int32_t r, double *__restrict__ t) {
    if (st->done) return;
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= r) return;
    double s = 0.0;
    for (int32_t b = 0; b < nb; ++b) s += partials[(size_t)b * r + q];
    t[q] = s;
}

// qv_j = sum_q F~_jq t_q + d~_j v_j
__global__ __launch_bounds__(kBlock) void k_qp_lowrank(const DevState *__restrict__ st, int32_t n,
                                                       const double *__restrict__ F, int32_t r,
                                                       const double *__restrict__ t,
                                                       const double *__restrict__ d,
                                                       const double *__restrict__ v,
                                                       double *__restrict__ qv) {
    if (st->done) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int32_t q = 0; q < r; ++q) acc = fma(F[(size_t)i * r + q], t[q], acc);
    qv[i] = acc + d[i] * v[i];
}

// qv = Q~ v, CSR rows with 8 lanes each
__global__ __launch_bounds__(kBlock) void k_qp_csr(const DevState *__restrict__ st, int32_t n,
                                                   const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const double *__restrict__ va,
                                                   const double *__restrict__ v,
                                                   double *__restrict__ qv) {
    if (st->done) return;
    const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 3;
    const int32_t lane = threadIdx.x & 7;
    double acc = 0.0;
    if (row < n)
        for (int32_t e = rp[row] + lane; e < rp[row + 1]; e += 8) acc = fma(va[e], v[ci[e]], acc);
    for (int off = 4; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (row < n && lane == 0) qv[row] = acc;
}

// qv = Q~ v, dense rows, one wave per row
__global__ __launch_bounds__(kBlock) void k_qp_dense(const DevState *__restrict__ st, int32_t n,
                                                     const double *__restrict__ Q,
                                                     const double *__restrict__ v,
                                                     double *__restrict__ qv) {
    if (st->done) return;
    const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int32_t lane = threadIdx.x & 63;
    double acc = 0.0;
    if (row < n)
        for (int32_t e = lane; e < n; e += 64) acc = fma(Q[(size_t)row * n + e], v[e], acc);
    acc = wave_sum(acc);
    if (row < n && lane == 0) qv[row] = acc;
}

__global__ __launch_bounds__(kBlock) void k_primal_qp(
    MatView M, const double *__restrict__ y, double *__restrict__ x, double *__restrict__ xbar,
    const double *__restrict__ qv, const double *__restrict__ c, const double *__restrict__ lv,
    const double *__restrict__ uv, double *__restrict__ xext, const DevState *__restrict__ st,
    int32_t j, double norm_q, double tau_override) {
    if (st->done) return;
    const RowSum rs = mat_row_dot(M, y);
    if (rs.valid) {
        const int32_t r = rs.row;
        const int64_t k = qp_k(st, j);
        const double theta = 2.0 / (double)(k + 2);
        const double tau = tau_override > 0.0
                               ? tau_override
                               : 1.0 / (st->omega / st->eta + 2.0 * norm_q / (double)(k + 1));
        const double xr = x[r];
        const double xp = clampd(xr - tau * (qv[r] + c[r] - rs.s), lv[r], uv[r]);
        xext[r] = 2.0 * xp - xr;
        x[r] = xp;
        xbar[r] = (1.0 - theta) * xbar[r] + theta * xp;
    }
}

__global__ __launch_bounds__(kBlock) void k_dual_qp(
    MatView M, const double *__restrict__ xext, double *__restrict__ y, double *__restrict__ ybar,
    const double *__restrict__ lc, const double *__restrict__ uc, const DevState *__restrict__ st,
    int32_t j, double sigma_override) {
    if (st->done) return;
    const RowSum rs = mat_row_dot(M, xext);
    if (rs.valid) {
        const int32_t r = rs.row;
        const int64_t k = qp_k(st, j);
        const double theta = 2.0 / (double)(k + 2);
        const double sigma = sigma_override > 0.0 ? sigma_override : st->sigma;
        const double yp = dual_prox(y[r], rs.s, sigma, lc[r], uc[r]);
        y[r] = yp;
        ybar[r] = (1.0 - theta) * ybar[r] + theta * yp;
    }
}

// Column side of a QP check on (xbar, ybar); qv = Q~ xbar. Sums:
//  0 |xbar - x0|^2  1 |r_d|^2  2 x'Qx  3 c'x  4 l_v'lambda^+ - u_v'lambda^- (original space)
// and the infeasibility-ray terms as for LPs (rays[4] per workgroup), the
// primal ray's violation also counting |(Q dx)_j| = |qv - Q~x0| / D_c; the
// products A~'ybar, Q~xbar are kept in qhat, qvhat.
__global__ __launch_bounds__(kBlock) void k_qp_check_n(
    MatView M, const double *__restrict__ ybar, const double *__restrict__ xbar,
    const double *__restrict__ x0, const double *__restrict__ qv, const double *__restrict__ Dc,
    const double *__restrict__ c_o, const double *__restrict__ lv_o,
    const double *__restrict__ uv_o, double *__restrict__ partials,
    const double *__restrict__ q0, double *__restrict__ qhat, const double *__restrict__ qv0,
    double *__restrict__ qvhat, double *__restrict__ rays, const DevState *__restrict__ st) {
    if (st->done) return;
    const RowSum rs = mat_row_dot(M, ybar);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double rsum[2] = {0.0, 0.0}, rmax[2] = {0.0, 0.0};
    if (rs.valid) {
        const int32_t r = rs.row;
        const double xb = xbar[r];
        const double d0 = xb - x0[r];
        v[0] = d0 * d0;
        const double d = Dc[r];
        const double xo = d * xb;
        const double qx = qv[r] / d;
        const double g = qx + c_o[r] - rs.s / d;
        const double lo = lv_o[r], hi = uv_o[r];
        const bool lf = isfinite(lo), uf = isfinite(hi);
        const double lam = (!lf && !uf) ? 0.0 : (lf && !uf) ? fmax(g, 0.0) : (!lf && uf) ? fmin(g, 0.0) : g;
        const double rd = g - lam;
        v[1] = rd * rd;
        v[2] = xo * qx;
        v[3] = c_o[r] * xo;
        v[4] = (lf ? lo * fmax(lam, 0.0) : 0.0) - (uf ? hi * fmax(-lam, 0.0) : 0.0);
        qhat[r] = rs.s;
        qvhat[r] = qv[r];
        ray_col_terms(rs.s, q0[r], d, d0, c_o[r], lo, hi, rsum, rmax);
        rmax[1] = fmax(rmax[1], fabs((qv[r] - qv0[r]) / d));
    }
    block_sum_store<6>(v, partials + (size_t)blockIdx.x * 6);
    block_sum_store<2>(rsum, rays + (size_t)blockIdx.x * 4);
    block_max_store<2>(rmax, rays + (size_t)blockIdx.x * 4 + 2);
}

// Row side: 0 |r_p|^2  1 l_c'y^+ - u_c'y^-  2 (unused)  3 |ybar - y0|^2
// (plus the rows' ray terms, rays[3] per workgroup; A~xbar kept in phat)
__global__ __launch_bounds__(kBlock) void k_qp_check_m(
    MatView M, const double *__restrict__ xbar, const double *__restrict__ ybar,
    const double *__restrict__ y0, const double *__restrict__ Dr, const double *__restrict__ lc_o,
    const double *__restrict__ uc_o, double *__restrict__ partials,
    const double *__restrict__ p0, double *__restrict__ phat, double *__restrict__ rays,
    const DevState *__restrict__ st) {
    if (st->done) return;
    const RowSum rs = mat_row_dot(M, xbar);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    double rsum[1] = {0.0}, rmax[2] = {0.0, 0.0};
    if (rs.valid) {
        const int32_t r = rs.row;
        const double d = Dr[r];
        const double ax = rs.s / d;
        const double lo = lc_o[r], hi = uc_o[r];
        const double rpr = ax - clampd(ax, lo, hi);
        v[0] = rpr * rpr;
        const double yb = ybar[r];
        const double yo = d * yb;
        v[1] = (isfinite(lo) ? lo * fmax(yo, 0.0) : 0.0) - (isfinite(hi) ? hi * fmax(-yo, 0.0) : 0.0);
        const double d0 = yb - y0[r];
        v[3] = d0 * d0;
        phat[r] = rs.s;
        ray_row_terms(rs.s, p0[r], d, d0, lo, hi, rsum, rmax);
    }
    block_sum_store<4>(v, partials + (size_t)blockIdx.x * 4);
    block_sum_store<1>(rsum, rays + (size_t)blockIdx.x * 3);
    block_max_store<2>(rmax, rays + (size_t)blockIdx.x * 3 + 1);
}

__global__ __launch_bounds__(kBlock) void k_qp_controller(
    DevState *__restrict__ st, const double *__restrict__ pn, int32_t nbn,
    const double *__restrict__ pm, int32_t nbm, const double *__restrict__ prn,
    const double *__restrict__ prm, CtlConst K, int32_t chunk_plain, int32_t is_last,
    int32_t last_status) {
    if (st->done) return;
    double vn[6], vm[4], rs[3], rx[2];
    const bool rays = K.detect && st->anchor_valid;
    check_totals(pn, nbn, pm, nbm, prn, prm, rays, vn, vm, rs, rx);
    if (threadIdx.x != 0) return;
    const int64_t t = st->t_next;
    const int64_t k = st->first ? 0 : st->k_base + st->plain_prev;
    const double P = 0.5 * vn[2] + vn[3];
    const double D = -0.5 * vn[2] + vm[1] + vn[4];
    const double abs_p = sqrt(vm[0]), abs_d = sqrt(vn[1]), abs_g = fabs(P - D);
    const double rel_p = abs_p / (1.0 + K.bnorm);
    const double rel_d = abs_d / (1.0 + K.cnorm);
    const double rel_g = abs_g / (1.0 + fabs(P) + fabs(D));
    double kkt = rel_p;
    if (rel_d > kkt || isnan(rel_d)) kkt = rel_d;
    if (rel_g > kkt || isnan(rel_g)) kkt = rel_g;
    st->kkt = kkt;
    st->rel_p = rel_p;
    st->rel_d = rel_d;
    st->rel_g = rel_g;
    st->pobj = P;
    st->dobj = D;
    st->abs_p = abs_p;
    st->abs_d = abs_d;
    st->abs_g = abs_g;
    st->k_check = k;
    st->t_done = t;
    st->first = 0;
    st->plain_prev = chunk_plain;
    st->t_next = t + 1 + chunk_plain;
    if (isnan(kkt)) {
        st->done = 1;
        st->status = PDHG_NUMERICAL_ERROR;
        st->action = 2;
        return;
    }
    if (kkt <= K.eps) {
        st->done = 1;
        st->status = PDHG_OPTIMAL;
        st->action = 2;
        return;
    }
    if (rays) {
        const double obj_d = rs[0] + rs[2], obj_p = rs[1];
        if (K.eps_pinf > 0.0 && obj_d > 0.0 && rx[0] <= K.eps_pinf * obj_d) {
            st->done = 1;
            st->status = PDHG_PRIMAL_INFEASIBLE;
            st->ray_scale = 1.0 / obj_d;
            st->action = 2;
            return;
        }
        if (K.eps_dinf > 0.0 && obj_p < 0.0 && rx[1] <= K.eps_dinf * (-obj_p)) {
            st->done = 1;
            st->status = PDHG_DUAL_INFEASIBLE;
            st->ray_scale = -1.0 / obj_p;
            st->action = 2;
            return;
        }
    }
    if (is_last) {
        st->done = 1;
        st->status = last_status;
        st->action = 2;
        return;
    }
    const double omega = st->omega;
    const double r = sqrt(omega * abs_p * abs_p + abs_d * abs_d / omega + abs_g * abs_g);
    st->last_r = r;
    int restart = 0;
    if (t == 0) {
        st->r_start = r;
        st->r_prev = r;
    } else if (r <= K.beta_suff * st->r_start ||
               (r <= K.beta_nec * st->r_start && r > st->r_prev) ||
               (double)k >= K.beta_art * (double)t) {
        restart = 1;
    } else {
        st->r_prev = r;
    }
    if (restart) {
        const double dxr = sqrt(vn[0]), dyr = sqrt(vm[3]);
        double w = omega;
        if (dxr > 1e-10 && dyr > 1e-10) w = exp(0.5 * log(dyr / dxr) + 0.5 * log(w));
        st->omega = w;
        st->tau = K.eta / w;
        st->sigma = K.eta * w;
        st->r_start = r;
        st->r_prev = r;
        st->restarts += 1;
        st->k_base = 0;
        st->action = 1;
        st->anchor_valid = 1;   // k_qp_apply stores the new anchor's products
    } else {
        st->k_base = k + 1;
        st->action = 0;
    }
}

// restart: x, x0 <- xbar and y, y0 <- ybar; the anchor's products A~'y0,
// Q~x0, A~x0 from this check's qhat, qvhat, phat
__global__ __launch_bounds__(kBlock) void k_qp_apply(const DevState *__restrict__ st, int32_t n,
                                                     int32_t m, double *__restrict__ x,
                                                     double *__restrict__ x0,
                                                     const double *__restrict__ xbar,
                                                     double *__restrict__ y, double *__restrict__ y0,
                                                     const double *__restrict__ ybar,
                                                     double *__restrict__ q0, const double *__restrict__ qhat,
                                                     double *__restrict__ qv0, const double *__restrict__ qvhat,
                                                     double *__restrict__ p0, const double *__restrict__ phat) {
    if (st->done || st->action != 1) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        x[i] = xbar[i];
        x0[i] = xbar[i];
        q0[i] = qhat[i];
        qv0[i] = qvhat[i];
    } else if (i - n < m) {
        const int64_t r = i - n;
        y[r] = ybar[r];
        y0[r] = ybar[r];
        p0[r] = phat[r];
    }
}

__global__ __launch_bounds__(kBlock) void k_copy2(int32_t n, int32_t m, const double *__restrict__ a,
                                                  double *__restrict__ b, const double *__restrict__ c,
                                                  double *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] = a[i];
    else if (i - n < m) d[i - n] = c[i - n];
}

// ---------------------------------------------------------------------------
// setup kernels

__global__ __launch_bounds__(kBlock) void k_qp_scale_lowrank(
    int32_t n, int32_t r, const int32_t *__restrict__ perm_c, const double *__restrict__ Dc,
    const double *__restrict__ F, const double *__restrict__ d, double *__restrict__ Fo,
    double *__restrict__ dout, int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t o = perm_c[i];
    const double dc = Dc[i];
    for (int32_t q = 0; q < r; ++q) {
        const double f = F[(size_t)o * r + q];
        if (!isfinite(f)) atomicOr(flag, 1);
        Fo[(size_t)i * r + q] = dc * f;
    }
    const double dd = d[o];
    if (!isfinite(dd)) atomicOr(flag, 1);
    dout[i] = (dc * dc) * dd;
}

__global__ __launch_bounds__(kBlock) void k_qp_scale_dense(int32_t n, const int32_t *__restrict__ perm_c,
                                                           const double *__restrict__ Dc,
                                                           const double *__restrict__ Q,
                                                           double *__restrict__ Qo,
                                                           int32_t *__restrict__ flag) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const int64_t i = t / n, j = t % n;
    const double q = Q[(size_t)perm_c[i] * n + perm_c[j]];
    if (!isfinite(q)) atomicOr(flag, 1);
    Qo[t] = (Dc[i] * q) * Dc[j];
}

// values of the permuted CSR Q (rows internal, columns internal): (D_i q) D_j
__global__ __launch_bounds__(kBlock) void k_qp_scale_csr(int32_t n, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         double *__restrict__ va,
                                                         const double *__restrict__ Dc) {
    const int64_t w = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= n) return;
    for (int32_t e = rp[w] + lane; e < rp[w + 1]; e += 64) va[e] = (Dc[w] * va[e]) * Dc[ci[e]];
}

__device__ __forceinline__ uint64_t splitmix64_q(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_qp_power_start(const int32_t *__restrict__ perm_c,
                                                           int32_t n, double *__restrict__ v,
                                                           double *__restrict__ partials) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double q[1] = {0.0};
    if (i < n) {
        const double val = 0.5 + (double)(splitmix64_q((uint64_t)perm_c[i]) >> 11) * 0x1.0p-53;
        v[i] = val;
        q[0] = val * val;
    }
    block_sum_store<1>(q, partials + blockIdx.x);
}

// partial sums of v'w and w'w
__global__ __launch_bounds__(kBlock) void k_qp_power_dots(const double *__restrict__ v,
                                                          const double *__restrict__ w, int32_t n,
                                                          double *__restrict__ partials) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double q[2] = {0.0, 0.0};
    if (i < n) {
        q[0] = v[i] * w[i];
        q[1] = w[i] * w[i];
    }
    block_sum_store<2>(q, partials + (size_t)blockIdx.x * 2);
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_qp_total(const double *__restrict__ partials, int32_t nb,
                                                     double *__restrict__ out) {
    double v[K];
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = 0.0;
    for (int32_t b = threadIdx.x; b < nb; b += kBlock)
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] += partials[(size_t)b * K + q];
    block_sum_all<K>(v);
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) out[q] = v[q];
}

// v = w / |w| and the history entry (lam = v'w with the previous v, |w|)
__global__ __launch_bounds__(kBlock) void k_qp_power_next(double *__restrict__ v,
                                                          const double *__restrict__ w, int32_t n,
                                                          const double *__restrict__ tot,
                                                          double *__restrict__ hist, int32_t it) {
    const double nw = sqrt(tot[1]);
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) {
        hist[2 * it] = tot[0];
        hist[2 * it + 1] = nw;
    }
    if (i < n && nw > 0.0) v[i] = w[i] / nw;
}

__global__ __launch_bounds__(kBlock) void k_qp_div(double *__restrict__ v, int32_t n,
                                                   const double *__restrict__ tot) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) v[i] = v[i] / sqrt(tot[0]);
}

// ---------------------------------------------------------------------------
// host side

static unsigned nblk(int64_t len) { return (unsigned)std::max<int64_t>(1, ceil_div(len, kBlock)); }

// qv = Q~ v with v from mode (0: momentum point with counter of step j, 1: xbar)
static void enqueue_qv(Handle &h, int32_t j, int32_t mode, const DevState *st) {
    hipStream_t s = h.stream;
    const int32_t n = h.n;
    const bool lr = h.q_kind == PDHG_FMT_LOWRANK_DIAG;
    k_qp_v<<<nblk(n), kBlock, 0, s>>>(st, n, j, mode, h.x.p, h.xbar.p, h.qv_in.p,
                                      lr ? h.q_f.p : nullptr, h.q_rank, h.qpart.p);
    if (lr) {
        k_qp_t<<<(unsigned)ceil_div(h.q_rank, 64), 64, 0, s>>>(st, h.qpart.p, (int32_t)nblk(n),
                                                               h.q_rank, h.qt.p);
        k_qp_lowrank<<<nblk(n), kBlock, 0, s>>>(st, n, h.q_f.p, h.q_rank, h.qt.p, h.q_d.p,
                                                h.qv_in.p, h.qv.p);
    } else if (h.q_kind == PDHG_FMT_CSR) {
        k_qp_csr<<<nblk((int64_t)n * 8), kBlock, 0, s>>>(st, n, h.q_rp.p, h.q_ci.p, h.q_va.p,
                                                         h.qv_in.p, h.qv.p);
    } else {
        k_qp_dense<<<nblk((int64_t)n * 64), kBlock, 0, s>>>(st, n, h.q_dense.p, h.qv_in.p, h.qv.p);
    }
}

void launch_qp_iteration(Handle &h, int32_t j) {
    enqueue_qv(h, j, 0, h.st.p);
    k_primal_qp<<<(unsigned)h.AT.nblocks(), kBlock, 0, h.stream>>>(
        view(h.AT), h.y.p, h.x.p, h.xbar.p, h.qv.p, h.c.p, h.lv.p, h.uv.p, h.xext.p, h.st.p, j,
        h.norm_q, -1.0);
    if (h.A.nblocks())
        k_dual_qp<<<(unsigned)h.A.nblocks(), kBlock, 0, h.stream>>>(
            view(h.A), h.xext.p, h.y.p, h.ybar.p, h.lc.p, h.uc.p, h.st.p, j, -1.0);
}

void launch_qp_check(Handle &h, int32_t chunk_plain, int32_t is_last, int32_t last_status) {
    hipStream_t s = h.stream;
    launch_qp_iteration(h, 0);
    enqueue_qv(h, 0, 1, h.st.p);
    k_qp_check_n<<<(unsigned)h.AT.nblocks(), kBlock, 0, s>>>(view(h.AT), h.ybar.p, h.xbar.p, h.x0.p,
                                                             h.qv.p, h.Dc.p, h.c_o.p, h.lv_o.p,
                                                             h.uv_o.p, h.pn.p, h.q0.p, h.qhat.p,
                                                             h.qv0.p, h.qvhat.p, h.prn.p, h.st.p);
    if (h.A.nblocks())
        k_qp_check_m<<<(unsigned)h.A.nblocks(), kBlock, 0, s>>>(view(h.A), h.xbar.p, h.ybar.p,
                                                               h.y0.p, h.Dr.p, h.lc_o.p, h.uc_o.p,
                                                               h.pm.p, h.p0.p, h.phat.p, h.prm.p,
                                                               h.st.p);
    CtlConst K;
    K.eps = h.opt.eps;
    K.bnorm = h.bnorm;
    K.cnorm = h.cnorm;
    K.eta = h.eta;
    K.beta_suff = h.opt.restart_sufficient;
    K.beta_nec = h.opt.restart_necessary;
    K.beta_art = h.opt.restart_artificial;
    K.norm_q = h.norm_q;
    K.qp = 1;
    K.detect = h.opt.eps_primal_infeasible > 0.0 || h.opt.eps_dual_infeasible > 0.0;
    K.eps_pinf = h.opt.eps_primal_infeasible;
    K.eps_dinf = h.opt.eps_dual_infeasible;
    K.term = 0;
    K.pad = 0;
    k_qp_controller<<<1, kBlock, 0, s>>>(h.st.p, h.pn.p, h.nbn, h.pm.p, h.nbm, h.prn.p, h.prm.p, K,
                                         chunk_plain, is_last, last_status);
    k_qp_apply<<<nblk((int64_t)h.n + h.m), kBlock, 0, s>>>(h.st.p, h.n, h.m, h.x.p, h.x0.p,
                                                          h.xbar.p, h.y.p, h.y0.p, h.ybar.p, h.q0.p,
                                                          h.qhat.p, h.qv0.p, h.qvhat.p, h.p0.p,
                                                          h.phat.p);
}

void launch_qp_init(Handle &h) {
    k_copy2<<<nblk((int64_t)h.n + h.m), kBlock, 0, h.stream>>>(h.n, h.m, h.x.p, h.xbar.p, h.y.p,
                                                              h.ybar.p);
}

void launch_qp_finalize(Handle &h, double *x_out, double *y_out) {
    if (h.n) launch_scatter_scaled(h.stream, h.perm_c.p, h.Dc.p, h.xbar.p, x_out, h.n);
    if (h.m) launch_scatter_scaled(h.stream, h.perm_r.p, h.Dr.p, h.ybar.p, y_out, h.m);
}

// one rAPDHG step with explicit k and omega (state already gathered into x, y, xbar, ybar)
void launch_qp_debug_step(Handle &h, int64_t k, double omega) {
    hipStream_t s = h.stream;
    // DevState with k_base = k and first = 0 so that step j = 1 uses counter k
    DevState ds;
    memset(&ds, 0, sizeof(ds));
    ds.eta = h.eta;
    ds.omega = omega;
    ds.tau = h.eta / omega;
    ds.sigma = h.eta * omega;
    ds.k_base = k;
    PDHG_HIP(hipMemcpyAsync(h.st.p, &ds, sizeof(ds), hipMemcpyHostToDevice, s));
    launch_qp_iteration(h, 1);
    PDHG_HIP(hipStreamSynchronize(s));
}

void qp_build(Handle &h, const pdhg_problem &p) {
    hipStream_t s = h.stream;
    const int32_t n = h.n;
    h.q_kind = p.q_format;
    DBuf<int32_t> flag;
    flag.alloc(1);
    PDHG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    auto dev_copy = [&](const void *src, size_t bytes, DBuf<uint8_t> &tmp) -> const void * {
        if (p.mem == PDHG_MEM_DEVICE) return src;
        tmp.alloc(bytes);
        PDHG_HIP(hipMemcpyAsync(tmp.p, src, bytes, hipMemcpyHostToDevice, s));
        return tmp.p;
    };
    DBuf<uint8_t> t1, t2, t3;
    if (h.q_kind == PDHG_FMT_LOWRANK_DIAG) {
        if (p.q_rank < 1 || p.q_rank > 4096 || !p.q_factor || !p.q_diag)
            fail(PDHG_ERR_INVALID_ARG, "low-rank Q needs 1 <= q_rank <= 4096, q_factor and q_diag");
        h.q_rank = p.q_rank;
        const double *F = (const double *)dev_copy(p.q_factor, sizeof(double) * (size_t)n * p.q_rank, t1);
        const double *d = (const double *)dev_copy(p.q_diag, sizeof(double) * (size_t)n, t2);
        h.q_f.alloc((size_t)n * h.q_rank);
        h.q_d.alloc(n);
        k_qp_scale_lowrank<<<nblk(n), kBlock, 0, s>>>(n, h.q_rank, h.perm_c.p, h.Dc.p, F, d, h.q_f.p,
                                                      h.q_d.p, flag.p);
        h.qpart.alloc((size_t)nblk(n) * h.q_rank);
        h.qt.alloc(h.q_rank);
    } else if (h.q_kind == PDHG_FMT_DENSE) {
        if (!p.q_dense) fail(PDHG_ERR_INVALID_ARG, "dense Q needs q_dense");
        if ((int64_t)n * n > ((int64_t)1 << 31)) fail(PDHG_ERR_UNSUPPORTED, "dense Q too large");
        const double *Q = (const double *)dev_copy(p.q_dense, sizeof(double) * (size_t)n * n, t1);
        h.q_dense.alloc((size_t)n * n);
        k_qp_scale_dense<<<nblk((int64_t)n * n), kBlock, 0, s>>>(n, h.perm_c.p, h.Dc.p, Q,
                                                                h.q_dense.p, flag.p);
        h.qpart.alloc(1);
    } else if (h.q_kind == PDHG_FMT_CSR) {
        if (!p.q_rowptr || (p.q_nnz > 0 && (!p.q_colidx || !p.q_val)) || p.q_nnz < 0 ||
            p.q_nnz >= INT32_MAX)
            fail(PDHG_ERR_INVALID_ARG, "bad CSR arrays for Q");
        const int32_t *qrp = (const int32_t *)dev_copy(p.q_rowptr, sizeof(int32_t) * ((size_t)n + 1), t1);
        const int32_t *qci = (const int32_t *)dev_copy(p.q_colidx, sizeof(int32_t) * (size_t)p.q_nnz, t2);
        const double *qva = (const double *)dev_copy(p.q_val, sizeof(double) * (size_t)p.q_nnz, t3);
        validate_csr(s, qrp, qci, qva, n, n, p.q_nnz);
        h.q_rp.alloc((size_t)n + 1);
        h.q_ci.alloc((size_t)p.q_nnz);
        h.q_va.alloc((size_t)p.q_nnz);
        permute_csr(s, n, n, p.q_nnz, qrp, qci, qva, h.perm_c.p, h.perm_c.p, h.q_rp.p, h.q_ci.p,
                    h.q_va.p);
        k_qp_scale_csr<<<nblk((int64_t)n * 64), kBlock, 0, s>>>(n, h.q_rp.p, h.q_ci.p, h.q_va.p,
                                                               h.Dc.p);
        h.qpart.alloc(1);
    } else {
        fail(PDHG_ERR_INVALID_ARG, "unknown q_format");
    }
    check_flag(s, flag.p, "non-finite entry in Q");
    h.xbar.alloc(n);
    h.ybar.alloc(std::max(1, h.m));
    h.qv_in.alloc(n);
    h.qv.alloc(n);
}

void qp_estimate_norm(Handle &h) {
    hipStream_t s = h.stream;
    const int32_t n = h.n;
    const int maxit = std::max(1, h.opt.power_max_iters);
    // the Q kernels check st->done: use a cleared state
    DevState ds;
    memset(&ds, 0, sizeof(ds));
    PDHG_HIP(hipMemcpyAsync(h.st.p, &ds, sizeof(ds), hipMemcpyHostToDevice, s));
    DBuf<double> part, tot, hist;
    part.alloc((size_t)nblk(n) * 2);
    tot.alloc(2);
    hist.alloc(2 * ((size_t)maxit + 2));
    // xbar holds v (mode 1 of enqueue_qv reads xbar)
    k_qp_power_start<<<nblk(n), kBlock, 0, s>>>(h.perm_c.p, n, h.xbar.p, part.p);
    k_qp_total<1><<<1, kBlock, 0, s>>>(part.p, (int32_t)nblk(n), tot.p);
    k_qp_div<<<nblk(n), kBlock, 0, s>>>(h.xbar.p, n, tot.p);
    std::vector<double> hh(2 * ((size_t)maxit + 2));
    double lam = 0.0, lam_prev = 0.0;
    bool stop = false;
    const int batch = 16;
    for (int it0 = 1; it0 <= maxit && !stop; it0 += batch) {
        const int it1 = std::min(maxit, it0 + batch - 1);
        for (int it = it0; it <= it1; ++it) {
            enqueue_qv(h, 0, 1, h.st.p);
            k_qp_power_dots<<<nblk(n), kBlock, 0, s>>>(h.xbar.p, h.qv.p, n, part.p);
            k_qp_total<2><<<1, kBlock, 0, s>>>(part.p, (int32_t)nblk(n), tot.p);
            k_qp_power_next<<<nblk(n), kBlock, 0, s>>>(h.xbar.p, h.qv.p, n, tot.p, hist.p, it);
        }
        PDHG_HIP(hipMemcpyAsync(hh.data() + 2 * it0, hist.p + 2 * it0,
                                sizeof(double) * 2 * (it1 - it0 + 1), hipMemcpyDeviceToHost, s));
        PDHG_HIP(hipStreamSynchronize(s));
        for (int it = it0; it <= it1; ++it) {
            lam = hh[2 * it];
            const double nw = hh[2 * it + 1];
            if (!(nw > 0.0)) {
                lam = 0.0;
                stop = true;
                break;
            }
            if (it > 1 && fabs(lam - lam_prev) <= h.opt.power_tol * fabs(lam)) {
                stop = true;
                break;
            }
            lam_prev = lam;
        }
    }
    h.norm_q = lam;
}

}  // namespace pdhg
