// Device-side helpers shared by the kernels: row mapping of the binned CSR
// layout, lane-group dot products and deterministic workgroup sums.
#pragma once

#include "common.hpp"

namespace pdhg {

constexpr int kSellUnroll = 8;   // SELL-64 entries whose loads are in flight together

struct RowCtx {
    int32_t row;
    int32_t lg;    // log2(lanes per row)
    bool valid;    // row exists
    bool lead;     // first lane of the row's lane group
};

// Workgroup blockIdx.x belongs to the last segment whose block_begin <= it.
__device__ __forceinline__ RowCtx row_ctx(const SegTable &T) {
    const int32_t b = blockIdx.x;
    int32_t si = 0;
#pragma unroll 1
    for (int32_t q = 1; q < T.nseg; ++q) si = (b >= T.s[q].block_begin) ? q : si;
    const int32_t lg = T.s[si].lanes_log2;
    RowCtx r;
    r.lg = lg;
    r.row = T.s[si].row_begin + (b - T.s[si].block_begin) * (kBlock >> lg) +
            (int32_t)(threadIdx.x >> lg);
    r.valid = r.row < T.s[si].row_end;
    r.lead = (threadIdx.x & ((1u << lg) - 1u)) == 0u;
    return r;
}

// sum_e val[e] * v[colidx[e]] over the row, lanes strided; the lane-group
// butterfly leaves the same total in every lane of the group.
__device__ __forceinline__ double row_dot(const int32_t *__restrict__ rowptr,
                                          const int32_t *__restrict__ colidx,
                                          const double *__restrict__ val,
                                          const double *__restrict__ v, const RowCtx &rc) {
    double acc = 0.0;
    const int32_t L = 1 << rc.lg;
    if (rc.valid) {
        const int32_t lane = (int32_t)(threadIdx.x & (uint32_t)(L - 1));
        const int32_t e1 = rowptr[rc.row + 1];
        for (int32_t e = rowptr[rc.row] + lane; e < e1; e += L)
            acc = fma(__builtin_nontemporal_load(&val[e]), v[__builtin_nontemporal_load(&colidx[e])], acc);
    }
    for (int32_t off = L >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    return acc;
}

// Row reduction of |val| (max when MAXNORM, else sum) without a vector.
template <bool MAXNORM>
__device__ __forceinline__ double row_absnorm(const int32_t *__restrict__ rowptr,
                                              const double *__restrict__ val, const RowCtx &rc) {
    double acc = 0.0;
    const int32_t L = 1 << rc.lg;
    if (rc.valid) {
        const int32_t lane = (int32_t)(threadIdx.x & (uint32_t)(L - 1));
        const int32_t e1 = rowptr[rc.row + 1];
        for (int32_t e = rowptr[rc.row] + lane; e < e1; e += L) {
            const double a = fabs(val[e]);
            acc = MAXNORM ? fmax(acc, a) : acc + a;
        }
    }
    for (int32_t off = L >> 1; off > 0; off >>= 1) {
        const double o = __shfl_xor(acc, off);
        acc = MAXNORM ? fmax(acc, o) : acc + o;
    }
    return acc;
}

struct RowSum {
    double s;
    int32_t row;
    bool valid;   // this thread owns an existing row and holds its full sum
};

// Index of the SELL-64 slice handled by this wave (wave-uniform), or -1 when
// the workgroup belongs to the long-row part.
__device__ __forceinline__ int32_t slice_of(const MatView &M) {
    if ((int32_t)blockIdx.x < M.seg.nblocks) return -1;
    return ((int32_t)blockIdx.x - M.seg.nblocks) * (kBlock / 64) + (int32_t)(threadIdx.x >> 6);
}

// acc + the products of entries [k, k + U) of a SELL-64 lane whose row has w
// entries (entry e at ci[64 e], va[64 e]; k < w, wave-uniform), in entry
// order. The loads are unconditional at indices clamped to the last entry, so
// the compiler issues all of them before the first product (with predicated
// loads it waits on each in turn); products of entries past w are dropped by a
// select, so the sum is exactly that of the entries < w.
template <int U, class Idx, class Gather>
__device__ __forceinline__ double sell_group(const Idx *__restrict__ ci,
                                             const double *__restrict__ va, int32_t k,
                                             int32_t w, double acc, Gather gather) {
    int32_t c[U];
    double a[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t e = 64 * min(k + u, w - 1);
        c[u] = (int32_t)__builtin_nontemporal_load(ci + e);
        a[u] = __builtin_nontemporal_load(va + e);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = gather(c[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const double t = fma(a[u], xv[u], acc);
        acc = (k + u < w) ? t : acc;
    }
    return acc;
}

// Sum of the w entries of a SELL-64 lane in entry order: groups of
// kSellUnroll, then one tail group of 1, 2, 4 or kSellUnroll (w is
// wave-uniform, so the group sizes are too).
template <class Idx, class Gather>
__device__ __forceinline__ double sell_lane_dot(const Idx *__restrict__ ci,
                                                const double *__restrict__ va, int32_t w,
                                                Gather gather) {
    double acc = 0.0;
    int32_t k = 0;
    for (; k + kSellUnroll <= w; k += kSellUnroll)
        acc = sell_group<kSellUnroll>(ci, va, k, w, acc, gather);
    const int32_t rest = w - k;
    if (rest > 4) acc = sell_group<kSellUnroll>(ci, va, k, w, acc, gather);
    else if (rest > 2) acc = sell_group<4>(ci, va, k, w, acc, gather);
    else if (rest == 2) acc = sell_group<2>(ci, va, k, w, acc, gather);
    else if (rest == 1) acc = sell_group<1>(ci, va, k, w, acc, gather);
    return acc;
}

// Row sum over SELL-64 slice sl (wave-uniform) for the row of this lane:
// entries walked in order with independent, coalesced loads.
__device__ __forceinline__ RowSum sell_row_dot(const MatView &M, const double *__restrict__ x,
                                               int32_t sl) {
    RowSum r;
    const int32_t lane = (int32_t)(threadIdx.x & 63);
    r.row = M.R_long + sl * 64 + lane;
    r.valid = sl < M.nslices && r.row < M.rows;
    double acc = 0.0;
    if (sl < M.nslices) {
        const int32_t b = __builtin_amdgcn_readfirstlane(M.slice_ptr[sl]);
        const int32_t w = (__builtin_amdgcn_readfirstlane(M.slice_ptr[sl + 1]) - b) >> 6;
        const int32_t *__restrict__ ci = M.colidx + b + lane;
        const double *__restrict__ va = M.val + b + lane;
        acc = sell_lane_dot(ci, va, w, [&](int32_t c) { return x[c]; });
    }
    r.s = acc;
    return r;
}

// Row sum of val * x[col] for the row owned by this thread (hybrid layout).
// Long rows: lane groups with a butterfly; short rows: one thread per row,
// entries walked in order with independent, coalesced loads.
__device__ __forceinline__ RowSum mat_row_dot(const MatView &M, const double *__restrict__ x) {
    const int32_t sl = slice_of(M);
    if (sl < 0) {
        RowSum r;
        const RowCtx rc = row_ctx(M.seg);
        r.s = row_dot(M.rowptr, M.colidx, M.val, x, rc);
        r.row = rc.row;
        r.valid = rc.valid && rc.lead;
        return r;
    }
    return sell_row_dot(M, x, sl);
}

// Row max (MAXNORM) or sum of |val| in the hybrid layout.
template <bool MAXNORM>
__device__ __forceinline__ RowSum mat_row_absnorm(const MatView &M) {
    RowSum r;
    const int32_t sl = slice_of(M);
    if (sl < 0) {
        const RowCtx rc = row_ctx(M.seg);
        r.s = row_absnorm<MAXNORM>(M.rowptr, M.val, rc);
        r.row = rc.row;
        r.valid = rc.valid && rc.lead;
        return r;
    }
    const int32_t lane = (int32_t)(threadIdx.x & 63);
    r.row = M.R_long + sl * 64 + lane;
    r.valid = sl < M.nslices && r.row < M.rows;
    double acc = 0.0;
    if (sl < M.nslices) {
        const int32_t b = M.slice_ptr[sl];
        const int32_t w = (M.slice_ptr[sl + 1] - b) >> 6;
        for (int32_t k = 0; k < w; ++k) {
            const double a = fabs(M.val[b + 64 * k + lane]);
            acc = MAXNORM ? fmax(acc, a) : acc + a;
        }
    }
    r.s = acc;
    return r;
}

// val <- val / (rfac[i] * cfac[j]) for every stored entry (i, j) of the rows
// of M; transposed: the rows of M are columns j and its column indices rows i.
// Padding entries hold 0.0 and stay 0.0.
__device__ __forceinline__ void mat_scale_entries(const MatView &M, const double *__restrict__ rfac,
                                                  const double *__restrict__ cfac, bool transposed) {
    const int32_t sl = slice_of(M);
    if (sl < 0) {
        const RowCtx rc = row_ctx(M.seg);
        if (!rc.valid) return;
        const int32_t L = 1 << rc.lg;
        const int32_t lane = (int32_t)(threadIdx.x & (uint32_t)(L - 1));
        for (int32_t e = M.rowptr[rc.row] + lane; e < M.rowptr[rc.row + 1]; e += L) {
            const int32_t o = M.colidx[e];
            const double ri = transposed ? rfac[o] : rfac[rc.row];
            const double sj = transposed ? cfac[rc.row] : cfac[o];
            M.val[e] = M.val[e] / (ri * sj);
        }
        return;
    }
    if (sl >= M.nslices) return;
    const int32_t lane = (int32_t)(threadIdx.x & 63);
    const int32_t row = M.R_long + sl * 64 + lane;
    if (row >= M.rows) return;
    const int32_t b = M.slice_ptr[sl];
    const int32_t w = (M.slice_ptr[sl + 1] - b) >> 6;
    for (int32_t k = 0; k < w; ++k) {
        const int32_t e = b + 64 * k + lane;
        const int32_t o = M.colidx[e];
        const double ri = transposed ? rfac[o] : rfac[row];
        const double sj = transposed ? cfac[row] : cfac[o];
        M.val[e] = M.val[e] / (ri * sj);
    }
}

__device__ __forceinline__ double wave_sum(double s) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    return s;
}

// Deterministic workgroup sum of K values per thread: wave butterflies, then
// the BT / 64 wave totals in fixed order (BT: threads of the workgroup).
// Result written by threads 0..K-1 to out.
template <int K, int BT = kBlock>
__device__ __forceinline__ void block_sum_store(const double (&v)[K], double *__restrict__ out) {
    __shared__ double sh[K][BT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) sh[q][wave] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < K) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < BT / 64; ++w) s += sh[threadIdx.x][w];
        out[threadIdx.x] = s;
    }
}

// Same, result broadcast to every thread.
template <int K>
__device__ __forceinline__ void block_sum_all(double (&v)[K]) {
    __shared__ double sh[K][kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) sh[q][wave] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += sh[q][w];
        v[q] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ double wave_max(double s) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off));
    return s;
}

// Workgroup maxima of K values per thread (order-free), written by threads
// 0..K-1 to out (BT: threads of the workgroup).
template <int K, int BT = kBlock>
__device__ __forceinline__ void block_max_store(const double (&v)[K], double *__restrict__ out) {
    __shared__ double sh[K][BT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double s = wave_max(v[q]);
        if (lane == 0) sh[q][wave] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < K) {
        double s = sh[threadIdx.x][0];
#pragma unroll
        for (int w = 1; w < BT / 64; ++w) s = fmax(s, sh[threadIdx.x][w]);
        out[threadIdx.x] = s;
    }
}

// Same, result broadcast to every thread.
template <int K>
__device__ __forceinline__ void block_max_all(double (&v)[K]) {
    __shared__ double sh[K][kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double s = wave_max(v[q]);
        if (lane == 0) sh[q][wave] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double s = sh[q][0];
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) s = fmax(s, sh[q][w]);
        v[q] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
    return fmin(fmax(v, lo), hi);
}

// Primal-weight update after a restart: log-smoothing (weight 1/2) towards
// |dy| / |dx|. Out of line on purpose: restarts are rare, and inlined into
// the persistent kernels the constants of exp / log would stay in vector
// registers across the whole iteration loop.
static __device__ __noinline__ double batch_new_omega(double omega, double dxr, double dyr) {
    if (dxr > 1e-10 && dyr > 1e-10) return exp(0.5 * log(dyr / dxr) + 0.5 * log(omega));
    return omega;
}

// Infeasibility-ray terms of one column j at a check, in the original space:
// q = (A~'yhat)_j, q0 = (A~'y0)_j, d = D_c[j], dxs = xhat_j - x0_j, c = c_j,
// [lo, hi] = [l_v, u_v]_j. With g = -(A'dy)_j and lam its part in the cone of
// the bounds: s[0] = l_v lam+ - u_v lam-, s[1] = c dx; mx[0] = |g - lam|,
// mx[1] = distance of dx to the recession cone of [l_v, u_v].
__device__ __forceinline__ void ray_col_terms(double q, double q0, double d, double dxs, double c,
                                              double lo, double hi, double (&s)[2], double (&mx)[2]) {
    const bool lf = isfinite(lo), uf = isfinite(hi);
    const double g = -(q - q0) / d;
    const double lam = (!lf && !uf) ? 0.0 : (lf && !uf) ? fmax(g, 0.0) : (!lf && uf) ? fmin(g, 0.0) : g;
    s[0] = (lf ? lo * fmax(lam, 0.0) : 0.0) - (uf ? hi * fmax(-lam, 0.0) : 0.0);
    mx[0] = fabs(g - lam);
    const double dx = d * dxs;
    s[1] = c * dx;
    mx[1] = fabs(dx - clampd(dx, lf ? 0.0 : -INFINITY, uf ? 0.0 : INFINITY));
}

// Same for row i: p = (A~xhat)_i, p0 = (A~x0)_i, d = D_r[i], dys = yhat_i -
// y0_i, [lo, hi] = [l_c, u_c]_i. With yp = proj_Y(dy): s[0] = l_c yp+ - u_c yp-;
// mx[0] = |dy - yp|, mx[1] = distance of (A dx)_i to the recession cone of
// [l_c, u_c].
__device__ __forceinline__ void ray_row_terms(double p, double p0, double d, double dys, double lo,
                                              double hi, double (&s)[1], double (&mx)[2]) {
    const bool lf = isfinite(lo), uf = isfinite(hi);
    const double dy = d * dys;
    const double yp = clampd(dy, uf ? -INFINITY : 0.0, lf ? INFINITY : 0.0);
    s[0] = (lf ? lo * fmax(yp, 0.0) : 0.0) - (uf ? hi * fmax(-yp, 0.0) : 0.0);
    mx[0] = fabs(dy - yp);
    const double a = (p - p0) / d;
    mx[1] = fabs(a - clampd(a, lf ? 0.0 : -INFINITY, uf ? 0.0 : INFINITY));
}

// Dual proximal step of eq. (pdhg-lp): v = y/sigma - a,
// yhat = sigma (v - proj_[-u_c, -l_c](v)); exactly 0 inside, exactly signed outside.
__device__ __forceinline__ double dual_prox(double y, double a, double sigma, double lc, double uc) {
    const double v = y / sigma - a;
    return sigma * (v - clampd(v, -uc, -lc));
}

// f(row) for the Q-value rows p[b * Q, b * Q + Q) of the blocks
// b = threadIdx.x + kBlock * i of one thread, in increasing b; eight blocks'
// loads are issued before their f calls.
template <int Q, class F>
__device__ __forceinline__ void strided_fold(const double *__restrict__ p, int32_t nb, F f) {
    int32_t b = (int32_t)threadIdx.x;
    for (; b + 7 * kBlock < nb; b += 8 * kBlock) {
        double t[8][Q];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int q = 0; q < Q; ++q) t[u][q] = p[(size_t)(b + u * kBlock) * Q + q];
#pragma unroll
        for (int u = 0; u < 8; ++u) f(t[u]);
    }
    for (; b < nb; b += kBlock) {
        double t[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) t[q] = p[(size_t)b * Q + q];
        f(t);
    }
}

// Totals of a check's per-workgroup partials, for the one-workgroup
// controllers (every thread ends with the same totals): vn / vm the six
// column-side and four row-side sums (pn: nbn rows of 6, pm: nbm rows of 4);
// with rays, rs the three ray sums (prn[b * 4 + 0, 1], prm[b * 3]) and rx the
// two ray maxima (prn[b * 4 + 2, 3] with prm[b * 3 + 1, 2]), else zeros.
__device__ __forceinline__ void check_totals(const double *__restrict__ pn, int32_t nbn,
                                             const double *__restrict__ pm, int32_t nbm,
                                             const double *__restrict__ prn,
                                             const double *__restrict__ prm, bool rays,
                                             double (&vn)[6], double (&vm)[4], double (&rs)[3],
                                             double (&rx)[2]) {
#pragma unroll
    for (int q = 0; q < 6; ++q) vn[q] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) vm[q] = 0.0;
    rs[0] = rs[1] = rs[2] = 0.0;
    rx[0] = rx[1] = 0.0;
    strided_fold<6>(pn, nbn, [&](const double *t) {
#pragma unroll
        for (int q = 0; q < 6; ++q) vn[q] += t[q];
    });
    strided_fold<4>(pm, nbm, [&](const double *t) {
#pragma unroll
        for (int q = 0; q < 4; ++q) vm[q] += t[q];
    });
    block_sum_all<6>(vn);
    block_sum_all<4>(vm);
    if (!rays) return;
    strided_fold<4>(prn, nbn, [&](const double *t) {
        rs[0] += t[0];
        rs[1] += t[1];
        rx[0] = fmax(rx[0], t[2]);
        rx[1] = fmax(rx[1], t[3]);
    });
    strided_fold<3>(prm, nbm, [&](const double *t) {
        rs[2] += t[0];
        rx[0] = fmax(rx[0], t[1]);
        rx[1] = fmax(rx[1], t[2]);
    });
    block_sum_all<3>(rs);
    block_max_all<2>(rx);
}

}  // namespace pdhg
