// Dense constraint matrices (row-major, m x n): the r2HPDHG iteration of
// eq. (pdhg-lp) / eq. (hrpdhg) with the two products done as HBM-streaming
// passes over A~ (FP64 GEMV has 0.25 flop per byte, far below the FP64 ridge,
// so the vector units keep up with HBM and matrix cores would not help):
//   rows pass    : a_i = A~_i . v, one wave per four rows (a workgroup per four
//                  rows when there are few), fused with the dual step
//   columns pass : partial sums of A~' w over 256-column tiles and row splits,
//                  then a finalize kernel that adds the splits in fixed order
//                  and applies the primal step.
// The epilogues repeat the formulas of the sparse kernels exactly.
#include "device.hpp"

namespace pdhg {

constexpr int kDenseSplits = 16;   // most row splits of the column pass
constexpr int kSplitRows = 256;    // fewest rows per split of the column pass

enum RowMode : int32_t {
    ROW_DUAL = 0,      // y <- Halpern(prox)
    ROW_DUAL_CHK = 1,  // yhat <- prox
    ROW_CHECK_M = 2,   // check sums over rows
    ROW_STORE_SQ = 3,  // out = a, partial sum of a^2
    ROW_ABSMAX = 4,    // out = max |A_i.|
    ROW_ABSSUM = 5     // out = sum |A_i.|
};

enum ColMode : int32_t {
    COL_PRIMAL = 0,
    COL_PRIMAL_CHK = 1,
    COL_CHECK_N = 2,
    COL_STORE_SQ = 3,
    COL_ABSMAX = 4,
    COL_ABSSUM = 5
};

struct DenseVecs {
    const double *x, *x0, *xhat, *aty, *c, *lv, *uv, *Dc, *c_o, *lv_o, *uv_o;
    double *xw, *xext, *xhat_w, *aty_w;
    const double *y, *y0, *yhat, *lc, *uc, *Dr, *lc_o, *uc_o;
    double *yw, *yhat_w;
    double *out, *partials;
    // checks: the anchor's products, this check's products, ray partials
    const double *p0, *q0;
    double *phat, *qhat, *rays;
    const DevState *st;
    int32_t j;
    double gamma, tau_o, sigma_o;
};

constexpr int kWideRows = 4;     // rows per workgroup of the WIDE row pass
constexpr int kWideBlock = 512;  // threads per workgroup of the WIDE row pass

// Row pass: a = sum_c A[i][c] v[c], or |A| norms. WIDE = false: one wave per
// four rows (lanes strided over the columns, each v[c] loaded once for the
// four rows, butterflies), sixteen rows per workgroup; WIDE = true: the whole
// workgroup on kWideRows rows (for few, long rows: enough loads in flight to
// stream HBM, each v[c] loaded once for them), wave totals added in wave order.
template <int MODE, bool WIDE>
__global__ __launch_bounds__(WIDE ? kWideBlock : kBlock) void k_dense_rows(
    const double *__restrict__ A, int32_t m, int32_t n, const double *__restrict__ v, DenseVecs d) {
    if (d.st && d.st->done) return;
    constexpr int BS = WIDE ? kWideBlock : kBlock;   // threads per workgroup
    constexpr int L = WIDE ? BS : 64;                 // lanes per row
    constexpr int R = WIDE ? kWideRows : 4;   // rows per workgroup (WIDE) or per wave
    const int64_t row0 = WIDE ? (int64_t)blockIdx.x * R
                              : (((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6) * R;
    const int32_t lane = WIDE ? (int32_t)threadIdx.x : (int32_t)(threadIdx.x & 63);
    double acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0;
    const double *__restrict__ Ar[R];
    bool live[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        live[q] = row0 + q < m;
        Ar[q] = A + (size_t)(live[q] ? row0 + q : 0) * n;
    }
    if (MODE == ROW_ABSMAX || MODE == ROW_ABSSUM) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (!live[q]) continue;
            for (int32_t c = lane; c < n; c += L) {
                const double a = fabs(Ar[q][c]);
                acc[q] = MODE == ROW_ABSMAX ? fmax(acc[q], a) : acc[q] + a;
            }
        }
    } else if (live[0]) {
        // U columns x R rows of independent loads in flight per lane, each
        // row added in column order
        constexpr int U = 16;
        int32_t c = lane;
        for (; c + (U - 1) * L < n; c += U * L) {
            double x[U], a[R][U];
#pragma unroll
            for (int k = 0; k < U; ++k) x[k] = v[c + k * L];
#pragma unroll
            for (int q = 0; q < R; ++q)
#pragma unroll
                for (int k = 0; k < U; ++k)
                    a[q][k] = live[q] ? __builtin_nontemporal_load(Ar[q] + c + k * L) : 0.0;
#pragma unroll
            for (int q = 0; q < R; ++q)
#pragma unroll
                for (int k = 0; k < U; ++k) acc[q] = fma(a[q][k], x[k], acc[q]);
        }
        for (; c < n; c += L) {
            const double x = v[c];
#pragma unroll
            for (int q = 0; q < R; ++q)
                if (live[q]) acc[q] = fma(__builtin_nontemporal_load(Ar[q] + c), x, acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (MODE == ROW_ABSMAX) {
            for (int off = 32; off > 0; off >>= 1) acc[q] = fmax(acc[q], __shfl_xor(acc[q], off));
        } else {
            acc[q] = wave_sum(acc[q]);
        }
    }
    double accv = acc[0];
    int64_t row = row0;
    if constexpr (WIDE) {
        // thread q of the workgroup owns row row0 + q
        __shared__ double wt[R][BS / 64];
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int q = 0; q < R; ++q) wt[q][threadIdx.x >> 6] = acc[q];
        }
        __syncthreads();
        const int32_t q = (int32_t)threadIdx.x;
        if (q < R) {
            double t = wt[q][0];
            for (int w = 1; w < BS / 64; ++w) t = MODE == ROW_ABSMAX ? fmax(t, wt[q][w]) : t + wt[q][w];
            accv = t;
        }
        row = row0 + (q < R ? q : 0);
    } else {
        // lane q of the wave owns row row0 + q
#pragma unroll
        for (int q = 1; q < R; ++q)
            if (lane == q) accv = acc[q];
        row = row0 + (lane < R ? lane : 0);
    }
    const double acc_own = accv;
    const bool own = row < m && (WIDE ? (int32_t)threadIdx.x < R : lane < R);
    if (MODE == ROW_CHECK_M || MODE == ROW_STORE_SQ) {
        double vals[4] = {0.0, 0.0, 0.0, 0.0};
        double rsum[1] = {0.0}, rmax[2] = {0.0, 0.0};
        if (own) {
            const int64_t r = row;
            if (MODE == ROW_STORE_SQ) {
                d.out[r] = acc_own;
                vals[0] = acc_own * acc_own;
            } else {
                const double dr = d.Dr[r];
                const double ax = acc_own / dr;
                const double lo = d.lc_o[r], hi = d.uc_o[r];
                const double rpr = ax - clampd(ax, lo, hi);
                vals[0] = rpr * rpr;
                const double yh = d.yhat[r];
                const double yo = dr * yh;
                vals[1] = (isfinite(lo) ? lo * fmax(yo, 0.0) : 0.0) - (isfinite(hi) ? hi * fmax(-yo, 0.0) : 0.0);
                const double dy = yh - d.y[r];
                vals[2] = dy * dy;
                const double d0 = yh - d.y0[r];
                vals[3] = d0 * d0;
                d.phat[r] = acc_own;
                ray_row_terms(acc_own, d.p0[r], dr, d0, lo, hi, rsum, rmax);
            }
        }
        if (MODE == ROW_STORE_SQ) {
            double q[1] = {vals[0]};
            block_sum_store<1, BS>(q, d.partials + blockIdx.x);
        } else {
            block_sum_store<4, BS>(vals, d.partials + (size_t)blockIdx.x * 4);
            block_sum_store<1, BS>(rsum, d.rays + (size_t)blockIdx.x * 3);
            block_max_store<2, BS>(rmax, d.rays + (size_t)blockIdx.x * 3 + 1);
        }
        return;
    }
    if (!own) return;
    const int64_t r = row;
    if (MODE == ROW_ABSMAX || MODE == ROW_ABSSUM) {
        d.out[r] = acc_own;
    } else if (MODE == ROW_DUAL) {
        const double sigma = d.st->sigma;
        const int64_t k = d.st->k_base + (d.j - 1);
        const double yr = d.y[r];
        const double yh = dual_prox(yr, acc_own, sigma, d.lc[r], d.uc[r]);
        const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
        d.yw[r] = ak * ((1.0 + d.gamma) * yh - d.gamma * yr) + bk * d.y0[r];
    } else if (MODE == ROW_DUAL_CHK) {
        const double sigma = d.sigma_o > 0.0 ? d.sigma_o : d.st->sigma;
        d.yhat_w[r] = dual_prox(d.y[r], acc_own, sigma, d.lc[r], d.uc[r]);
    }
}

// Partial column sums: partials[split][c] = sum over the split's rows of A[i][c] w[i];
// the splits are gridDim.y equal runs of rows.
template <bool ABSMAX, bool ABSSUM>
__global__ __launch_bounds__(kBlock) void k_dense_cols_partial(const double *__restrict__ A,
                                                               int32_t m, int32_t n,
                                                               const double *__restrict__ w,
                                                               double *__restrict__ partials,
                                                               const DevState *__restrict__ st) {
    if (st && st->done) return;
    const int64_t col = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int32_t split = blockIdx.y;
    const int32_t splits = (int32_t)gridDim.y;
    const int32_t rows_per = (m + splits - 1) / splits;
    const int32_t r0 = split * rows_per, r1 = min(m, r0 + rows_per);
    if (col >= n) return;
    double acc = 0.0;
    const double *__restrict__ Ac = A + col;
    int32_t i = r0;
    if (ABSMAX || ABSSUM) {
        for (; i < r1; ++i) {
            const double a = fabs(Ac[(size_t)i * n]);
            acc = ABSMAX ? fmax(acc, a) : acc + a;
        }
    } else {
        // sixteen, then eight rows' loads in flight per thread, added in row order
        for (; i + 15 < r1; i += 16) {
            double a[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) a[u] = __builtin_nontemporal_load(Ac + (size_t)(i + u) * n);
#pragma unroll
            for (int u = 0; u < 16; ++u) acc = fma(a[u], w[i + u], acc);
        }
        for (; i + 7 < r1; i += 8) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = __builtin_nontemporal_load(Ac + (size_t)(i + u) * n);
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = fma(a[u], w[i + u], acc);
        }
        for (; i < r1; ++i) acc = fma(__builtin_nontemporal_load(Ac + (size_t)i * n), w[i], acc);
    }
    partials[(size_t)split * n + col] = acc;
}

// Splits added in order 0..S-1, then the column epilogue.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_dense_cols_final(int32_t n, int32_t splits,
                                                             const double *__restrict__ part,
                                                             DenseVecs d) {
    if (d.st && d.st->done) return;
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double s = 0.0;
    if (r < n) {
        for (int q = 0; q < splits; ++q) {
            const double p = part[(size_t)q * n + r];
            s = MODE == COL_ABSMAX ? fmax(s, p) : s + p;
        }
    }
    if (MODE == COL_CHECK_N || MODE == COL_STORE_SQ) {
        double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double rsum[2] = {0.0, 0.0}, rmax[2] = {0.0, 0.0};
        if (r < n) {
            if (MODE == COL_STORE_SQ) {
                d.out[r] = s;
                v[0] = s * s;
            } else {
                const double q = s;
                const double xh = d.xhat[r];
                const double dx = xh - d.x[r];
                v[0] = dx * dx;
                v[1] = (q - d.aty[r]) * dx;
                const double d0 = xh - d.x0[r];
                v[2] = d0 * d0;
                const double dd = d.Dc[r];
                const double xo = dd * xh;
                const double g = d.c_o[r] - q / dd;
                const double lo = d.lv_o[r], hi = d.uv_o[r];
                const bool lf = isfinite(lo), uf = isfinite(hi);
                const double lam = (!lf && !uf) ? 0.0 : (lf && !uf) ? fmax(g, 0.0) : (!lf && uf) ? fmin(g, 0.0) : g;
                const double rd = g - lam;
                v[3] = rd * rd;
                v[4] = d.c_o[r] * xo;
                v[5] = (lf ? lo * fmax(lam, 0.0) : 0.0) - (uf ? hi * fmax(-lam, 0.0) : 0.0);
                d.qhat[r] = q;
                ray_col_terms(q, d.q0[r], dd, d0, d.c_o[r], lo, hi, rsum, rmax);
            }
        }
        if (MODE == COL_STORE_SQ) {
            double q1[1] = {v[0]};
            block_sum_store<1>(q1, d.partials + blockIdx.x);
        } else {
            block_sum_store<6>(v, d.partials + (size_t)blockIdx.x * 6);
            block_sum_store<2>(rsum, d.rays + (size_t)blockIdx.x * 4);
            block_max_store<2>(rmax, d.rays + (size_t)blockIdx.x * 4 + 2);
        }
        return;
    }
    if (r >= n) return;
    if (MODE == COL_ABSMAX || MODE == COL_ABSSUM) {
        d.out[r] = s;
    } else if (MODE == COL_PRIMAL) {
        const double tau = d.st->tau;
        const int64_t k = d.st->k_base + (d.j - 1);
        const double xr = d.x[r];
        const double xh = clampd(xr - tau * (d.c[r] - s), d.lv[r], d.uv[r]);
        const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
        d.xext[r] = 2.0 * xh - xr;
        d.xw[r] = ak * ((1.0 + d.gamma) * xh - d.gamma * xr) + bk * d.x0[r];
    } else if (MODE == COL_PRIMAL_CHK) {
        const double tau = d.tau_o > 0.0 ? d.tau_o : d.st->tau;
        const double xr = d.x[r];
        const double xh = clampd(xr - tau * (d.c[r] - s), d.lv[r], d.uv[r]);
        d.xhat_w[r] = xh;
        d.xext[r] = 2.0 * xh - xr;
        d.aty_w[r] = s;
    }
}

// A~_ij <- A~_ij / (r_i s_j) elementwise; also finite check of the input.
__global__ __launch_bounds__(kBlock) void k_dense_scale(double *__restrict__ A, int32_t m, int32_t n,
                                                        const double *__restrict__ rf,
                                                        const double *__restrict__ cf) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t total = (int64_t)m * n;
    for (int64_t e = t; e < total; e += (int64_t)gridDim.x * kBlock) {
        const int64_t i = e / n, j = e - i * n;
        A[e] = A[e] / (rf[i] * cf[j]);
    }
}

__global__ __launch_bounds__(kBlock) void k_dense_finite(const double *__restrict__ A, int64_t total,
                                                         int32_t *__restrict__ flag) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int64_t e = t; e < total; e += (int64_t)gridDim.x * kBlock)
        if (!isfinite(A[e])) atomicOr(flag, 2);
}

__global__ __launch_bounds__(kBlock) void k_iota(int32_t *__restrict__ p, int32_t len) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) p[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// host side

static unsigned dblk(int64_t len) { return (unsigned)std::max<int64_t>(1, ceil_div(len, kBlock)); }

static DenseVecs dvecs(Handle &h, int32_t j) {
    DenseVecs d;
    memset(&d, 0, sizeof(d));
    d.x = h.x.p;
    d.x0 = h.x0.p;
    d.xhat = h.xhat.p;
    d.aty = h.aty.p;
    d.c = h.c.p;
    d.lv = h.lv.p;
    d.uv = h.uv.p;
    d.Dc = h.Dc.p;
    d.c_o = h.c_o.p;
    d.lv_o = h.lv_o.p;
    d.uv_o = h.uv_o.p;
    d.xw = h.x.p;
    d.xext = h.xext.p;
    d.xhat_w = h.xhat.p;
    d.aty_w = h.aty.p;
    d.y = h.y.p;
    d.y0 = h.y0.p;
    d.yhat = h.yhat.p;
    d.lc = h.lc.p;
    d.uc = h.uc.p;
    d.Dr = h.Dr.p;
    d.lc_o = h.lc_o.p;
    d.uc_o = h.uc_o.p;
    d.yw = h.y.p;
    d.yhat_w = h.yhat.p;
    d.st = h.st.p;
    d.j = j;
    d.gamma = h.opt.gamma;
    d.tau_o = -1.0;
    d.sigma_o = -1.0;
    return d;
}

// Few rows (fewer than 4 per CU) get a workgroup each, otherwise a wave per four.
static bool wide_rows(int32_t m) { return m < 1024; }
static unsigned row_blocks(int32_t m) {
    return wide_rows(m) ? (unsigned)std::max<int64_t>(1, ceil_div(m, kWideRows)) : dblk((int64_t)(m + 3) / 4 * 64);
}

template <int MODE>
static void launch_rows(hipStream_t s, const double *A, int32_t m, int32_t n, const double *v,
                        const DenseVecs &d) {
    if (wide_rows(m))
        k_dense_rows<MODE, true><<<row_blocks(m), kWideBlock, 0, s>>>(A, m, n, v, d);
    else
        k_dense_rows<MODE, false><<<row_blocks(m), kBlock, 0, s>>>(A, m, n, v, d);
}
static unsigned col_blocks(int32_t n) { return dblk(n); }
// Row splits of the column pass: up to kDenseSplits, at least kSplitRows rows each.
static int32_t col_splits(int32_t m) {
    return (int32_t)std::min<int64_t>(kDenseSplits, std::max<int64_t>(1, m / kSplitRows));
}

int32_t dense_row_blocks(const Handle &h) { return (int32_t)row_blocks(h.m); }
int32_t dense_col_blocks(const Handle &h) { return (int32_t)col_blocks(h.n); }

static void cols_partial(Handle &h, const double *w, const DevState *st) {
    dim3 grid(col_blocks(h.n), col_splits(h.m));
    k_dense_cols_partial<false, false><<<grid, kBlock, 0, h.stream>>>(h.Ad.p, h.m, h.n, w, h.dpart.p, st);
}

void dense_primal(Handle &h, int32_t j) {
    cols_partial(h, h.y.p, h.st.p);
    k_dense_cols_final<COL_PRIMAL><<<col_blocks(h.n), kBlock, 0, h.stream>>>(h.n, col_splits(h.m), h.dpart.p, dvecs(h, j));
}

void dense_dual(Handle &h, int32_t j) {
    if (h.m == 0) return;
    launch_rows<ROW_DUAL>(h.stream, h.Ad.p, h.m, h.n, h.xext.p, dvecs(h, j));
}

void dense_primal_check(Handle &h, double tau_override) {
    cols_partial(h, h.y.p, h.st.p);
    DenseVecs d = dvecs(h, 0);
    d.tau_o = tau_override;
    k_dense_cols_final<COL_PRIMAL_CHK><<<col_blocks(h.n), kBlock, 0, h.stream>>>(h.n, col_splits(h.m), h.dpart.p, d);
}

void dense_dual_check(Handle &h, double sigma_override) {
    if (h.m == 0) return;
    DenseVecs d = dvecs(h, 0);
    d.sigma_o = sigma_override;
    launch_rows<ROW_DUAL_CHK>(h.stream, h.Ad.p, h.m, h.n, h.xext.p, d);
}

void dense_check_sums(Handle &h) {
    cols_partial(h, h.yhat.p, h.st.p);
    DenseVecs d = dvecs(h, 0);
    d.partials = h.pn.p;
    d.q0 = h.q0.p;
    d.qhat = h.qhat.p;
    d.rays = h.prn.p;
    k_dense_cols_final<COL_CHECK_N><<<col_blocks(h.n), kBlock, 0, h.stream>>>(h.n, col_splits(h.m), h.dpart.p, d);
    if (h.m > 0) {
        DenseVecs e = dvecs(h, 0);
        e.partials = h.pm.p;
        e.p0 = h.p0.p;
        e.phat = h.phat.p;
        e.rays = h.prm.p;
        launch_rows<ROW_CHECK_M>(h.stream, h.Ad.p, h.m, h.n, h.xhat.p, e);
    }
}

// out = A~ v with partial sums of out^2 (rows), for the power iteration
void dense_rows_sq(Handle &h, const double *v, double *out, double *partials) {
    DenseVecs d = dvecs(h, 0);
    d.st = nullptr;
    d.out = out;
    d.partials = partials;
    launch_rows<ROW_STORE_SQ>(h.stream, h.Ad.p, h.m, h.n, v, d);
}

// out = A~' w with partial sums of out^2 (columns)
void dense_cols_sq(Handle &h, const double *w, double *out, double *partials) {
    cols_partial(h, w, nullptr);
    DenseVecs d = dvecs(h, 0);
    d.st = nullptr;
    d.out = out;
    d.partials = partials;
    k_dense_cols_final<COL_STORE_SQ><<<col_blocks(h.n), kBlock, 0, h.stream>>>(h.n, col_splits(h.m), h.dpart.p, d);
}

void dense_build(Handle &h, const pdhg_problem &p) {
    hipStream_t s = h.stream;
    const int64_t total = (int64_t)h.m * h.n;
    h.Ad.alloc((size_t)std::max<int64_t>(1, total));
    if (total > 0)
        PDHG_HIP(hipMemcpyAsync(h.Ad.p, p.a_dense, sizeof(double) * (size_t)total,
                                p.mem == PDHG_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                         : hipMemcpyHostToDevice,
                                s));
    DBuf<int32_t> flag;
    flag.alloc(1);
    PDHG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    if (total > 0) k_dense_finite<<<4096, kBlock, 0, s>>>(h.Ad.p, total, flag.p);
    check_flag(s, flag.p, "non-finite entry in the dense matrix");
    h.perm_r.alloc(h.m);
    h.perm_c.alloc(h.n);
    if (h.m) k_iota<<<dblk(h.m), kBlock, 0, s>>>(h.perm_r.p, h.m);
    k_iota<<<dblk(h.n), kBlock, 0, s>>>(h.perm_c.p, h.n);
    h.dpart.alloc((size_t)kDenseSplits * h.n);
    h.A.rows = h.m;
    h.A.cols = h.n;
    h.A.nnz = total;
    h.AT.rows = h.n;
    h.AT.cols = h.m;
    h.AT.nnz = total;
    PDHG_HIP(hipStreamSynchronize(s));
}

void dense_scale(Handle &h) {
    hipStream_t s = h.stream;
    const int32_t m = h.m, n = h.n;
    DBuf<double> rn, cn;
    rn.alloc(m);
    cn.alloc(n);
    const int passes = h.opt.ruiz_iters + (h.opt.pock_chambolle ? 1 : 0);
    for (int pass = 0; pass < passes && m > 0; ++pass) {
        const bool pc = pass >= h.opt.ruiz_iters;
        DenseVecs d = dvecs(h, 0);
        d.st = nullptr;
        d.out = rn.p;
        dim3 grid(col_blocks(n), col_splits(m));
        if (pc) {
            launch_rows<ROW_ABSSUM>(s, h.Ad.p, m, n, nullptr, d);
            k_dense_cols_partial<false, true><<<grid, kBlock, 0, s>>>(h.Ad.p, m, n, nullptr, h.dpart.p, nullptr);
            d.out = cn.p;
            k_dense_cols_final<COL_ABSSUM><<<col_blocks(n), kBlock, 0, s>>>(n, col_splits(m), h.dpart.p, d);
        } else {
            launch_rows<ROW_ABSMAX>(s, h.Ad.p, m, n, nullptr, d);
            k_dense_cols_partial<true, false><<<grid, kBlock, 0, s>>>(h.Ad.p, m, n, nullptr, h.dpart.p, nullptr);
            d.out = cn.p;
            k_dense_cols_final<COL_ABSMAX><<<col_blocks(n), kBlock, 0, s>>>(n, col_splits(m), h.dpart.p, d);
        }
        launch_factors(h, rn.p, cn.p);
        k_dense_scale<<<8192, kBlock, 0, s>>>(h.Ad.p, m, n, rn.p, cn.p);
    }
    PDHG_HIP(hipStreamSynchronize(s));
}

}  // namespace pdhg
