// r2HPDHG iteration kernels (MPAX paper, Algorithm 1 with eq. (pdhg-lp) and
// eq. (hrpdhg)), all in the scaled space and internal order.
//
// Plain iteration = two launches:
//   primal: s = A~'y (rows of A'), xhat = clamp(x - tau (c - s)), writes
//           xext = 2 xhat - x and the Halpern point x <- a_k((1+g) xhat - g x) + b_k x0
//   dual:   a = A~ xext (rows of A), yhat = dual prox, writes the Halpern point y.
// Check iteration (every check_every steps) = primal/dual variants that keep
// (xhat, yhat), two extra products A~'yhat and A~ xhat fused with the KKT and
// fixed-point-residual sums, a one-workgroup controller and an apply kernel.
#include "device.hpp"

namespace pdhg {

// Primal update of row r given s = (A~'y)_r: PDHG point, extrapolation and
// the Halpern step (Algorithm 1). The row's vector entries are loaded first
// (PrimalIn), before the product they do not depend on.
struct PrimalIn {
    double x, x0, c, lv, uv;
};
__device__ __forceinline__ PrimalIn primal_load(int32_t r, const double *__restrict__ x,
                                                const double *__restrict__ x0,
                                                const double *__restrict__ c,
                                                const double *__restrict__ lv,
                                                const double *__restrict__ uv) {
    return PrimalIn{x[r], x0[r], c[r], lv[r], uv[r]};
}
__device__ __forceinline__ void primal_store(int32_t r, double s, const PrimalIn &in,
                                             double *__restrict__ x, double *__restrict__ xext,
                                             const DevState *st, int32_t j, double gamma) {
    const double tau = st->tau;
    const int64_t k = st->k_base + (j - 1);
    const double xh = clampd(in.x - tau * (in.c - s), in.lv, in.uv);
    const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
    xext[r] = 2.0 * xh - in.x;
    x[r] = ak * ((1.0 + gamma) * xh - gamma * in.x) + bk * in.x0;
}
__device__ __forceinline__ void primal_update(int32_t r, double s, double *__restrict__ x,
                                              const double *__restrict__ x0,
                                              const double *__restrict__ c,
                                              const double *__restrict__ lv,
                                              const double *__restrict__ uv,
                                              double *__restrict__ xext, const DevState *st,
                                              int32_t j, double gamma) {
    primal_store(r, s, primal_load(r, x, x0, c, lv, uv), x, xext, st, j, gamma);
}

// Check-iteration primal step of row r given s = (A~'y)_r: the PDHG point
// xhat, xext = 2 xhat - x, and s kept for the checks.
__device__ __forceinline__ void primal_chk_store(int32_t r, double s, const double *__restrict__ x,
                                                 const double *__restrict__ c,
                                                 const double *__restrict__ lv,
                                                 const double *__restrict__ uv,
                                                 double *__restrict__ xhat, double *__restrict__ xext,
                                                 double *__restrict__ aty, const DevState *st,
                                                 double tau_override) {
    const double tau = tau_override > 0.0 ? tau_override : st->tau;
    const double xr = x[r];
    const double xh = clampd(xr - tau * (c[r] - s), lv[r], uv[r]);
    xhat[r] = xh;
    xext[r] = 2.0 * xh - xr;
    aty[r] = s;
}

// Dual update of row r given a = (A~ xext)_r: dual prox and the Halpern step.
struct DualIn {
    double y, y0, lc, uc;
};
__device__ __forceinline__ DualIn dual_load(int32_t r, const double *__restrict__ y,
                                            const double *__restrict__ y0,
                                            const double *__restrict__ lc,
                                            const double *__restrict__ uc) {
    return DualIn{y[r], y0[r], lc[r], uc[r]};
}
__device__ __forceinline__ void dual_store(int32_t r, double a, const DualIn &in,
                                           double *__restrict__ y, const DevState *st, int32_t j,
                                           double gamma) {
    const double sigma = st->sigma;
    const int64_t k = st->k_base + (j - 1);
    const double yh = dual_prox(in.y, a, sigma, in.lc, in.uc);
    const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
    y[r] = ak * ((1.0 + gamma) * yh - gamma * in.y) + bk * in.y0;
}
__device__ __forceinline__ void dual_update(int32_t r, double a, double *__restrict__ y,
                                            const double *__restrict__ y0,
                                            const double *__restrict__ lc,
                                            const double *__restrict__ uc, const DevState *st,
                                            int32_t j, double gamma) {
    dual_store(r, a, dual_load(r, y, y0, lc, uc), y, st, j, gamma);
}

__global__ __launch_bounds__(kBlock) void k_primal(
    MatView M, const double *__restrict__ y, double *__restrict__ x,
    const double *__restrict__ x0, const double *__restrict__ c, const double *__restrict__ lv,
    const double *__restrict__ uv, double *__restrict__ xext, const DevState *__restrict__ st,
    int32_t j, double gamma) {
    if (st->done) return;
    const RowSum rs = mat_row_dot(M, y);
    if (rs.valid) primal_update(rs.row, rs.s, x, x0, c, lv, uv, xext, st, j, gamma);
}

__global__ __launch_bounds__(kBlock) void k_dual(
    MatView M, const double *__restrict__ xext, double *__restrict__ y,
    const double *__restrict__ y0, const double *__restrict__ lc, const double *__restrict__ uc,
    const DevState *__restrict__ st, int32_t j, double gamma) {
    if (st->done) return;
    const RowSum rs = mat_row_dot(M, xext);
    if (rs.valid) dual_update(rs.row, rs.s, y, y0, lc, uc, st, j, gamma);
}

// Primal step over the SELL-64 slices [skip, nslices) of A~' (the rows before
// them go through the LDS panels).
__global__ __launch_bounds__(kBlock) void k_primal_sell(
    MatView M, int32_t skip, const double *__restrict__ y, double *__restrict__ x,
    const double *__restrict__ x0, const double *__restrict__ c, const double *__restrict__ lv,
    const double *__restrict__ uv, double *__restrict__ xext, const DevState *__restrict__ st,
    int32_t j, double gamma) {
    if (st->done) return;
    const int32_t sl = skip + (int32_t)blockIdx.x * (kBlock / 64) + (int32_t)(threadIdx.x >> 6);
    const int32_t r = M.R_long + sl * 64 + (int32_t)(threadIdx.x & 63);
    const bool valid = sl < M.nslices && r < M.rows;
    PrimalIn in{};
    if (valid) in = primal_load(r, x, x0, c, lv, uv);
    const RowSum rs = sell_row_dot(M, y, sl);
    if (valid) primal_store(r, rs.s, in, x, xext, st, j, gamma);
}

// sh[0, len) = src[0, len) for a kPanelThreads workgroup (len <= N):
// every load of a thread is issued before the first LDS store, then the
// workgroup synchronises.
template <int N = kPanelMax>
__device__ __forceinline__ void stage_lds(double *sh, const double *__restrict__ src, int32_t len) {
    constexpr int kPer = N / kPanelThreads;
    double t[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int32_t i = (int32_t)threadIdx.x + u * kPanelThreads;
        t[u] = i < len ? src[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int32_t i = (int32_t)threadIdx.x + u * kPanelThreads;
        if (i < len) sh[i] = t[u];
    }
    __syncthreads();
}

// Piece sums of the LDS panels (PanelMat). The workgroup stages its panel of
// v in LDS; its waves take the panel's SELL-64 slices round robin (the widest
// first), one lane per piece, entries summed in order by sell_lane_dot; the
// next slice's bounds and slots are loaded while the current one is reduced.
__global__ __launch_bounds__(kPanelThreads) void k_panel_dot(PanelView P,
                                                             const double *__restrict__ v,
                                                             const DevState *__restrict__ st) {
    if (st->done) return;
    const int32_t p = P.wg_panel[blockIdx.x];
    if (p < 0) return;
    __shared__ double sh[kPanelMax];
    const int32_t base = p * P.S;
    stage_lds(sh, v + base, min(P.S, P.vlen - base));
    const int32_t wave = (int32_t)(threadIdx.x >> 6), lane = (int32_t)(threadIdx.x & 63);
    const int32_t s1 = P.pslice[p + 1];
    const int32_t stride = P.W * kPanelWaves;
    int32_t sl = P.pslice[p] + P.wg_rank[blockIdx.x] * kPanelWaves + wave;
    if (sl >= s1) return;
    int32_t nb = P.soff[sl], ne = P.soff[sl + 1], nslot = P.slot[(size_t)sl * 64 + lane];
    while (sl < s1) {
        const int32_t b = __builtin_amdgcn_readfirstlane(nb);
        const int32_t w = (__builtin_amdgcn_readfirstlane(ne) - b) >> 6;
        const int32_t slot = nslot;
        const int32_t nx = min(sl + stride, s1 - 1);
        nb = P.soff[nx];
        ne = P.soff[nx + 1];
        nslot = P.slot[(size_t)nx * 64 + lane];
        const uint16_t *__restrict__ ip = P.idx + b + lane;
        const double *__restrict__ vp = P.val + b + lane;
        const double acc = sell_lane_dot(ip, vp, w, [&](int32_t c) { return sh[c]; });
        if (slot >= 0) P.part[slot] = acc;
        sl += stride;
    }
}

// (A~'v)_r for a panel row: the first pieces of its sub-rows in panel order
// (all lanes read panel p together), then its further pieces.
__device__ __forceinline__ double panel_sum(const PanelView &P, int32_t r) {
    double s = 0.0;
    for (int32_t w = 0; w < P.W64; ++w) {
        const uint64_t mk = P.mask[(size_t)w * P.R + r];
        const int32_t pe = min(64, P.P - 64 * w);
        const double *__restrict__ col = P.part + (size_t)(64 * w) * P.R + r;
        int32_t b = 0;
        for (; b + 16 <= pe; b += 16) {
            double t[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) t[u] = ((mk >> (b + u)) & 1ull) ? col[(size_t)(b + u) * P.R] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if ((mk >> (b + u)) & 1ull) s += t[u];
        }
        for (; b < pe; ++b)
            if ((mk >> b) & 1ull) s += col[(size_t)b * P.R];
    }
    for (int32_t e = P.xptr[r]; e < P.xptr[r + 1]; ++e) s += P.part[P.xslot[e]];
    return s;
}

// Primal step of the panel rows [0, R) of A~'.
__global__ __launch_bounds__(kBlock) void k_primal_panels(
    PanelView P, double *__restrict__ x, const double *__restrict__ x0,
    const double *__restrict__ c, const double *__restrict__ lv, const double *__restrict__ uv,
    double *__restrict__ xext, const DevState *__restrict__ st, int32_t j, double gamma) {
    if (st->done) return;
    const int32_t r = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (r >= P.R) return;
    const PrimalIn in = primal_load(r, x, x0, c, lv, uv);
    primal_store(r, panel_sum(P, r), in, x, xext, st, j, gamma);
}

// The check iteration's primal step in the panel layout: k_primal_sell and
// k_primal_panels with the check epilogue (primal_chk_store).
__global__ __launch_bounds__(kBlock) void k_primal_sell_chk(
    MatView M, int32_t skip, const double *__restrict__ y, const double *__restrict__ x,
    const double *__restrict__ c, const double *__restrict__ lv, const double *__restrict__ uv,
    double *__restrict__ xhat, double *__restrict__ xext, double *__restrict__ aty,
    const DevState *__restrict__ st, double tau_override) {
    if (st->done) return;
    const int32_t sl = skip + (int32_t)blockIdx.x * (kBlock / 64) + (int32_t)(threadIdx.x >> 6);
    const int32_t r = M.R_long + sl * 64 + (int32_t)(threadIdx.x & 63);
    const bool valid = sl < M.nslices && r < M.rows;
    const RowSum rs = sell_row_dot(M, y, sl);
    if (valid) primal_chk_store(r, rs.s, x, c, lv, uv, xhat, xext, aty, st, tau_override);
}

__global__ __launch_bounds__(kBlock) void k_primal_panels_chk(
    PanelView P, const double *__restrict__ x, const double *__restrict__ c,
    const double *__restrict__ lv, const double *__restrict__ uv, double *__restrict__ xhat,
    double *__restrict__ xext, double *__restrict__ aty, const DevState *__restrict__ st,
    double tau_override) {
    if (st->done) return;
    const int32_t r = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (r >= P.R) return;
    primal_chk_store(r, panel_sum(P, r), x, c, lv, uv, xhat, xext, aty, st, tau_override);
}

// Dual step over the SELL-64 slices of A~ with x_ext[0, H) staged in LDS
// (columns are sorted by length, so these are the most gathered entries).
// Persistent workgroups take the slices round robin. The sums are formed in
// the same order as sell_row_dot, so the result equals k_dual's bit for bit.
__global__ __launch_bounds__(kPanelThreads) void k_dual_hot(
    MatView M, int32_t H, const double *__restrict__ xext, double *__restrict__ y,
    const double *__restrict__ y0, const double *__restrict__ lc, const double *__restrict__ uc,
    const DevState *__restrict__ st, int32_t j, double gamma) {
    if (st->done) return;
    __shared__ double sh[kHotMax];
    stage_lds<kHotMax>(sh, xext, H);
    const int32_t lane = (int32_t)(threadIdx.x & 63);
    const int32_t nw = (int32_t)gridDim.x * kPanelWaves;
    int32_t sl = (int32_t)blockIdx.x * kPanelWaves + (int32_t)(threadIdx.x >> 6);
    if (sl >= M.nslices) return;
    // the next slice's bounds are loaded while the current one is reduced
    int32_t nb = M.slice_ptr[sl], ne = M.slice_ptr[sl + 1];
    while (sl < M.nslices) {
        const int32_t b = __builtin_amdgcn_readfirstlane(nb);
        const int32_t w = (__builtin_amdgcn_readfirstlane(ne) - b) >> 6;
        const int32_t nx = min(sl + nw, M.nslices - 1);
        nb = M.slice_ptr[nx];
        ne = M.slice_ptr[nx + 1];
        const int32_t *__restrict__ ci = M.colidx + b + lane;
        const double *__restrict__ va = M.val + b + lane;
        const int32_t r = M.R_long + sl * 64 + lane;
        DualIn in{};
        if (r < M.rows) in = dual_load(r, y, y0, lc, uc);
        const double acc = sell_lane_dot(ci, va, w, [&](int32_t c) { return c < H ? sh[c] : xext[c]; });
        if (r < M.rows) dual_store(r, acc, in, y, st, j, gamma);
        sl += nw;
    }
}

// Step sizes and inner counter of a debug iteration.
__global__ void k_set_step(DevState *st, double tau, double sigma, int64_t k) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->tau = tau;
    st->sigma = sigma;
    st->k_base = k;
}

__global__ __launch_bounds__(kBlock) void k_primal_chk(
    MatView M, const double *__restrict__ y, const double *__restrict__ x,
    const double *__restrict__ c, const double *__restrict__ lv, const double *__restrict__ uv,
    double *__restrict__ xhat, double *__restrict__ xext, double *__restrict__ aty,
    const DevState *__restrict__ st, double tau_override) {
    if (st->done) return;
    const RowSum rs = mat_row_dot(M, y);
    if (rs.valid) primal_chk_store(rs.row, rs.s, x, c, lv, uv, xhat, xext, aty, st, tau_override);
}

__global__ __launch_bounds__(kBlock) void k_dual_chk(
    MatView M, const double *__restrict__ xext, const double *__restrict__ y,
    const double *__restrict__ lc, const double *__restrict__ uc, double *__restrict__ yhat,
    const DevState *__restrict__ st, double sigma_override) {
    if (st->done) return;
    const RowSum rs = mat_row_dot(M, xext);
    const double a = rs.s;
    if (rs.valid) {
        const int32_t r = rs.row;
        const double sigma = sigma_override > 0.0 ? sigma_override : st->sigma;
        yhat[r] = dual_prox(y[r], a, sigma, lc[r], uc[r]);
    }
}

// Column side of a check: q = A~'yhat. Sums (per workgroup):
//  0 |xhat - x|^2   1 (q - A~'y)'(xhat - x)   2 |xhat - x0|^2
//  3 |r_d|^2 (original space)   4 c'x (original)   5 l_v'lambda^+ - u_v'lambda^-
// Rays from the anchor (original space; dx = D_c (xhat - x0), g = -A'dy with
// A'dy = (q - A~'y0) / D_c), per workgroup into rays[4]: sums of the dual
// ray's l_v'lam+ - u_v'lam- and of c'dx, maxima of |g - lam| and of the
// distance of dx to the recession cone of [l_v, u_v]. q is kept in qhat.
// Column side of a check for row r of A~' given q = (A~'yhat)_r (see k_check_n).
__device__ __forceinline__ void check_n_terms(
    int32_t r, double q, const double *__restrict__ xhat, const double *__restrict__ x,
    const double *__restrict__ x0, const double *__restrict__ aty, const double *__restrict__ Dc,
    const double *__restrict__ c_o, const double *__restrict__ lv_o, const double *__restrict__ uv_o,
    const double *__restrict__ q0, double *__restrict__ qhat, double (&v)[6], double (&rsum)[2],
    double (&rmax)[2]) {
    const double xh = xhat[r];
    const double dx = xh - x[r];
    v[0] = dx * dx;
    v[1] = (q - aty[r]) * dx;
    const double d0 = xh - x0[r];
    v[2] = d0 * d0;
    const double d = Dc[r];
    const double xo = d * xh;
    const double g = c_o[r] - q / d;
    const double lo = lv_o[r], hi = uv_o[r];
    const bool lf = isfinite(lo), uf = isfinite(hi);
    const double lam = (!lf && !uf) ? 0.0 : (lf && !uf) ? fmax(g, 0.0) : (!lf && uf) ? fmin(g, 0.0) : g;
    const double rd = g - lam;
    v[3] = rd * rd;
    v[4] = c_o[r] * xo;
    v[5] = (lf ? lo * fmax(lam, 0.0) : 0.0) - (uf ? hi * fmax(-lam, 0.0) : 0.0);
    qhat[r] = q;
    ray_col_terms(q, q0[r], d, d0, c_o[r], lo, hi, rsum, rmax);
}

__global__ __launch_bounds__(kBlock) void k_check_n(
    MatView M, const double *__restrict__ yhat, const double *__restrict__ xhat,
    const double *__restrict__ x, const double *__restrict__ x0, const double *__restrict__ aty,
    const double *__restrict__ Dc, const double *__restrict__ c_o, const double *__restrict__ lv_o,
    const double *__restrict__ uv_o, double *__restrict__ partials,
    const double *__restrict__ q0, double *__restrict__ qhat, double *__restrict__ rays,
    const DevState *__restrict__ st) {
    if (st->done) return;
    const RowSum rs = mat_row_dot(M, yhat);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double rsum[2] = {0.0, 0.0}, rmax[2] = {0.0, 0.0};
    if (rs.valid)
        check_n_terms(rs.row, rs.s, xhat, x, x0, aty, Dc, c_o, lv_o, uv_o, q0, qhat, v, rsum, rmax);
    block_sum_store<6>(v, partials + (size_t)blockIdx.x * 6);
    block_sum_store<2>(rsum, rays + (size_t)blockIdx.x * 4);
    block_max_store<2>(rmax, rays + (size_t)blockIdx.x * 4 + 2);
}

// The column side of a check in the panel layout: the SELL-64 rows from slice
// skip on (workgroup b writes block b of the partials), and the panel rows
// [0, R) (workgroup b writes block b0 + b), each with k_check_n's terms.
__global__ __launch_bounds__(kBlock) void k_check_n_sell(
    MatView M, int32_t skip, const double *__restrict__ yhat, const double *__restrict__ xhat,
    const double *__restrict__ x, const double *__restrict__ x0, const double *__restrict__ aty,
    const double *__restrict__ Dc, const double *__restrict__ c_o, const double *__restrict__ lv_o,
    const double *__restrict__ uv_o, double *__restrict__ partials,
    const double *__restrict__ q0, double *__restrict__ qhat, double *__restrict__ rays,
    const DevState *__restrict__ st) {
    if (st->done) return;
    const int32_t sl = skip + (int32_t)blockIdx.x * (kBlock / 64) + (int32_t)(threadIdx.x >> 6);
    const int32_t r = M.R_long + sl * 64 + (int32_t)(threadIdx.x & 63);
    const bool valid = sl < M.nslices && r < M.rows;
    const RowSum rs = sell_row_dot(M, yhat, sl);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double rsum[2] = {0.0, 0.0}, rmax[2] = {0.0, 0.0};
    if (valid) check_n_terms(r, rs.s, xhat, x, x0, aty, Dc, c_o, lv_o, uv_o, q0, qhat, v, rsum, rmax);
    block_sum_store<6>(v, partials + (size_t)blockIdx.x * 6);
    block_sum_store<2>(rsum, rays + (size_t)blockIdx.x * 4);
    block_max_store<2>(rmax, rays + (size_t)blockIdx.x * 4 + 2);
}

__global__ __launch_bounds__(kBlock) void k_check_n_panels(
    PanelView P, int32_t b0, const double *__restrict__ xhat, const double *__restrict__ x,
    const double *__restrict__ x0, const double *__restrict__ aty, const double *__restrict__ Dc,
    const double *__restrict__ c_o, const double *__restrict__ lv_o, const double *__restrict__ uv_o,
    double *__restrict__ partials, const double *__restrict__ q0, double *__restrict__ qhat,
    double *__restrict__ rays, const DevState *__restrict__ st) {
    if (st->done) return;
    const int32_t r = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double rsum[2] = {0.0, 0.0}, rmax[2] = {0.0, 0.0};
    if (r < P.R)
        check_n_terms(r, panel_sum(P, r), xhat, x, x0, aty, Dc, c_o, lv_o, uv_o, q0, qhat, v, rsum, rmax);
    const size_t b = (size_t)b0 + blockIdx.x;
    block_sum_store<6>(v, partials + b * 6);
    block_sum_store<2>(rsum, rays + b * 4);
    block_max_store<2>(rmax, rays + b * 4 + 2);
}

// Row side of a check: p = A~ xhat. Sums:
//  0 |r_p|^2 (original)   1 l_c'y^+ - u_c'y^-   2 |yhat - y|^2   3 |yhat - y0|^2
// Rays from the anchor (dy = D_r (yhat - y0), A dx = (p - A~x0) / D_r), per
// workgroup into rays[3]: the sum of l_c'yp+ - u_c'yp- for yp = proj_Y(dy),
// maxima of |dy - yp| and of the distance of A dx to the recession cone of
// [l_c, u_c]. p is kept in phat.
__global__ __launch_bounds__(kBlock) void k_check_m(
    MatView M, const double *__restrict__ xhat, const double *__restrict__ yhat,
    const double *__restrict__ y, const double *__restrict__ y0, const double *__restrict__ Dr,
    const double *__restrict__ lc_o, const double *__restrict__ uc_o, double *__restrict__ partials,
    const double *__restrict__ p0, double *__restrict__ phat, double *__restrict__ rays,
    const DevState *__restrict__ st) {
    if (st->done) return;
    const RowSum rs = mat_row_dot(M, xhat);
    const double p = rs.s;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    double rsum[1] = {0.0}, rmax[2] = {0.0, 0.0};
    if (rs.valid) {
        const int32_t r = rs.row;
        const double d = Dr[r];
        const double ax = p / d;
        const double lo = lc_o[r], hi = uc_o[r];
        const double rpr = ax - clampd(ax, lo, hi);
        v[0] = rpr * rpr;
        const double yh = yhat[r];
        const double yo = d * yh;
        v[1] = (isfinite(lo) ? lo * fmax(yo, 0.0) : 0.0) - (isfinite(hi) ? hi * fmax(-yo, 0.0) : 0.0);
        const double dy = yh - y[r];
        v[2] = dy * dy;
        const double d0 = yh - y0[r];
        v[3] = d0 * d0;
        phat[r] = p;
        ray_row_terms(p, p0[r], d, d0, lo, hi, rsum, rmax);
    }
    block_sum_store<4>(v, partials + (size_t)blockIdx.x * 4);
    block_sum_store<1>(rsum, rays + (size_t)blockIdx.x * 3);
    block_max_store<2>(rmax, rays + (size_t)blockIdx.x * 3 + 1);
}

// One workgroup: totals of the check sums in fixed order, relative KKT error,
// fixed-point residual in the PDHG norm, termination and restart decisions,
// primal-weight update.
__global__ __launch_bounds__(kBlock) void k_controller(
    DevState *__restrict__ st, const double *__restrict__ pn, int32_t nbn,
    const double *__restrict__ pm, int32_t nbm, const double *__restrict__ prn,
    const double *__restrict__ prm, CtlConst K, int32_t chunk_plain, int32_t is_last,
    int32_t last_status) {
    if (st->done) return;
    double vn[6], vm[4], rs[3], rx[2];
    // ray totals: 0 dual-ray objective (columns), 1 c'dx, 2 dual-ray objective
    // (rows); maxima: 0 dual-ray violation, 1 primal-ray violation
    const bool rays = K.detect && st->anchor_valid;
    check_totals(pn, nbn, pm, nbm, prn, prm, rays, vn, vm, rs, rx);
    if (threadIdx.x != 0) return;

    const int64_t t = st->t_next;
    const int64_t k = st->first ? 0 : st->k_base + st->plain_prev;
    const double P = vn[4];
    const double D = vm[1] + vn[5];
    const double abs_p = sqrt(vm[0]), abs_d = sqrt(vn[3]), abs_g = fabs(P - D);
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
    // a polishing phase stops on its own residual alone
    const double term_val = K.term == 1 ? rel_p : K.term == 2 ? rel_d : kkt;
    if (term_val <= K.eps) {
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
    const double tau = st->tau, sigma = st->sigma;
    double r2 = vn[0] / tau + vm[2] / sigma + 2.0 * vn[1];
    const double r = r2 > 0.0 ? sqrt(r2) : 0.0;
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
        const double dxr = sqrt(vn[2]), dyr = sqrt(vm[3]);
        double omega = st->omega;
        if (dxr > 1e-10 && dyr > 1e-10) omega = exp(0.5 * log(dyr / dxr) + 0.5 * log(omega));
        st->omega = omega;
        st->tau = K.eta / omega;
        st->sigma = K.eta * omega;
        st->r_start = r;
        st->r_prev = r;
        st->restarts += 1;
        st->k_base = 0;
        st->action = 1;
        st->anchor_valid = 1;   // k_apply stores the new anchor's products
    } else {
        st->k_base = k + 1;
        st->action = 0;
    }
}

// Restart (z <- zhat, anchor <- zhat) or Halpern step at the check iteration.
// With q0 / p0 set, a restart also stores the anchor's products A~'y0, A~x0
// (the check's qhat, phat) for the infeasibility rays.
__global__ __launch_bounds__(kBlock) void k_apply(
    const DevState *__restrict__ st, int32_t n, int32_t m, double *__restrict__ x,
    double *__restrict__ x0, const double *__restrict__ xhat, double *__restrict__ y,
    double *__restrict__ y0, const double *__restrict__ yhat, double gamma,
    double *__restrict__ q0, const double *__restrict__ qhat, double *__restrict__ p0,
    const double *__restrict__ phat) {
    if (st->done) return;
    const int32_t act = st->action;
    const int64_t k = st->k_check;
    const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double xh = xhat[i];
        if (act == 1) {
            x[i] = xh;
            x0[i] = xh;
            if (q0) q0[i] = qhat[i];
        } else {
            x[i] = ak * ((1.0 + gamma) * xh - gamma * x[i]) + bk * x0[i];
        }
    } else if (i - n < m) {
        const int64_t r = i - n;
        const double yh = yhat[r];
        if (act == 1) {
            y[r] = yh;
            y0[r] = yh;
            if (p0) p0[r] = phat[r];
        } else {
            y[r] = ak * ((1.0 + gamma) * yh - gamma * y[r]) + bk * y0[r];
        }
    }
}

// Halpern point of a debug step with an explicit inner counter.
__global__ __launch_bounds__(kBlock) void k_halpern_explicit(
    int32_t n, int32_t m, int64_t k, const double *__restrict__ x, const double *__restrict__ x0,
    const double *__restrict__ xhat, const double *__restrict__ y, const double *__restrict__ y0,
    const double *__restrict__ yhat, double *__restrict__ xn, double *__restrict__ yn,
    double gamma) {
    const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        xn[i] = ak * ((1.0 + gamma) * xhat[i] - gamma * x[i]) + bk * x0[i];
    } else if (i - n < m) {
        const int64_t r = i - n;
        yn[r] = ak * ((1.0 + gamma) * yhat[r] - gamma * y[r]) + bk * y0[r];
    }
}

// Initial point: x = proj_X(x_init / D_c), y = proj_Y(y_init / D_r) (zeros when
// no warm start), anchors equal to it.
__global__ __launch_bounds__(kBlock) void k_init_point(
    int32_t n, int32_t m, const int32_t *__restrict__ perm_c, const int32_t *__restrict__ perm_r,
    const double *__restrict__ x_init, const double *__restrict__ y_init,
    const double *__restrict__ Dc, const double *__restrict__ Dr, const double *__restrict__ lv,
    const double *__restrict__ uv, const double *__restrict__ lc, const double *__restrict__ uc,
    double *__restrict__ x, double *__restrict__ x0, double *__restrict__ y,
    double *__restrict__ y0) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double v = x_init ? x_init[perm_c[i]] / Dc[i] : 0.0;
        const double xv = clampd(v, lv[i], uv[i]);
        x[i] = xv;
        x0[i] = xv;
    } else if (i - n < m) {
        const int64_t r = i - n;
        const double v = y_init ? y_init[perm_r[r]] / Dr[r] : 0.0;
        const double lo = isfinite(uc[r]) ? -INFINITY : 0.0;
        const double hi = isfinite(lc[r]) ? INFINITY : 0.0;
        const double yv = clampd(v, lo, hi);
        y[r] = yv;
        y0[r] = yv;
    }
}

__global__ void k_reset_state(DevState *st, double eta, double omega) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    DevState s;
    memset(&s, 0, sizeof(s));
    s.eta = eta;
    s.omega = omega;
    s.tau = eta / omega;
    s.sigma = eta * omega;
    s.first = 1;
    s.status = PDHG_UNSOLVED;
    *st = s;
}

__global__ __launch_bounds__(kBlock) void k_gather(const int32_t *__restrict__ perm,
                                                   const double *__restrict__ src,
                                                   double *__restrict__ dst, int32_t len) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) dst[i] = src[perm[i]];
}

__global__ __launch_bounds__(kBlock) void k_scatter(const int32_t *__restrict__ perm,
                                                    const double *__restrict__ src,
                                                    double *__restrict__ dst, int32_t len) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) dst[perm[i]] = src[i];
}

__global__ __launch_bounds__(kBlock) void k_scatter_scaled(const int32_t *__restrict__ perm,
                                                           const double *__restrict__ scale,
                                                           const double *__restrict__ src,
                                                           double *__restrict__ dst, int32_t len) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) dst[perm[i]] = scale[i] * src[i];
}

// ---------------------------------------------------------------------------
// host wrappers

static inline dim3 grid_of(const HMat &M) { return dim3((unsigned)M.nblocks()); }

void launch_primal(Handle &h, int32_t j, hipEvent_t *timing) {
    // timing: four events; [0, 1] and [2, 3] bracket the step's kernels on the
    // stream(s) they run on (one stream: [0] before, [1..3] after)
    auto one_stream = [&](bool before) {
        if (!timing) return;
        if (before) {
            PDHG_HIP(hipEventRecord(timing[0], h.stream));
        } else {
            PDHG_HIP(hipEventRecord(timing[1], h.stream));
            PDHG_HIP(hipEventRecord(timing[2], h.stream));
            PDHG_HIP(hipEventRecord(timing[3], h.stream));
        }
    };
    if (h.dense || h.AT.nblocks() == 0) {
        one_stream(true);
        if (h.dense) dense_primal(h, j);
        one_stream(false);
        return;
    }
    if (h.PT.R > 0) {
        // panel rows on stream2 beside the SELL-64 rest on the main stream;
        // timing (4 events): around the kernels on stream2, then on the main stream
        PDHG_HIP(hipEventRecord(h.ev_fork, h.stream));
        PDHG_HIP(hipStreamWaitEvent(h.stream2, h.ev_fork, 0));
        const PanelView P = view(h.PT);
        if (timing) PDHG_HIP(hipEventRecord(timing[0], h.stream2));
        k_panel_dot<<<h.PT.nwg, kPanelThreads, 0, h.stream2>>>(P, h.y.p, h.st.p);
        k_primal_panels<<<(unsigned)ceil_div(h.PT.R, kBlock), kBlock, 0, h.stream2>>>(
            P, h.x.p, h.x0.p, h.c.p, h.lv.p, h.uv.p, h.xext.p, h.st.p, j, h.opt.gamma);
        if (timing) PDHG_HIP(hipEventRecord(timing[1], h.stream2));
        PDHG_HIP(hipEventRecord(h.ev_join, h.stream2));
        const int32_t ns = h.AT.nslices - h.sell_skip;
        if (timing) PDHG_HIP(hipEventRecord(timing[2], h.stream));
        if (ns > 0)
            k_primal_sell<<<(unsigned)ceil_div(ns, kBlock / 64), kBlock, 0, h.stream>>>(
                view(h.AT), h.sell_skip, h.y.p, h.x.p, h.x0.p, h.c.p, h.lv.p, h.uv.p, h.xext.p,
                h.st.p, j, h.opt.gamma);
        if (timing) PDHG_HIP(hipEventRecord(timing[3], h.stream));
        PDHG_HIP(hipStreamWaitEvent(h.stream, h.ev_join, 0));
        return;
    }
    one_stream(true);
    k_primal<<<grid_of(h.AT), kBlock, 0, h.stream>>>(
        view(h.AT), h.y.p, h.x.p, h.x0.p, h.c.p, h.lv.p,
        h.uv.p, h.xext.p, h.st.p, j, h.opt.gamma);
    one_stream(false);
}

void launch_dual(Handle &h, int32_t j) {
    if (h.dense) {
        dense_dual(h, j);
        return;
    }
    if (h.A.nblocks() == 0) return;
    if (h.hot_cols > 0) {
        // long rows (lane groups) by the standard kernel, SELL-64 slices by the hot one
        if (h.A.seg.nblocks > 0)
            k_dual<<<(unsigned)h.A.seg.nblocks, kBlock, 0, h.stream>>>(
                view(h.A), h.xext.p, h.y.p, h.y0.p, h.lc.p, h.uc.p, h.st.p, j, h.opt.gamma);
        if (h.A.nslices > 0)
            k_dual_hot<<<(unsigned)h.dual_wgs, kPanelThreads, 0, h.stream>>>(
                view(h.A), h.hot_cols, h.xext.p, h.y.p, h.y0.p, h.lc.p, h.uc.p, h.st.p, j,
                h.opt.gamma);
        return;
    }
    k_dual<<<grid_of(h.A), kBlock, 0, h.stream>>>(view(h.A), h.xext.p, h.y.p, h.y0.p, h.lc.p,
                                                  h.uc.p, h.st.p, j, h.opt.gamma);
}

void launch_set_step(Handle &h, double tau, double sigma, int64_t k) {
    k_set_step<<<1, 1, 0, h.stream>>>(h.st.p, tau, sigma, k);
}

void launch_primal_check(Handle &h, double tau_override) {
    if (h.dense) {
        dense_primal_check(h, tau_override);
        return;
    }
    if (h.AT.nblocks() == 0) return;
    if (h.PT.R > 0) {
        // as launch_primal: the panel rows on stream2 beside the SELL-64 rest
        PDHG_HIP(hipEventRecord(h.ev_fork, h.stream));
        PDHG_HIP(hipStreamWaitEvent(h.stream2, h.ev_fork, 0));
        const PanelView P = view(h.PT);
        k_panel_dot<<<h.PT.nwg, kPanelThreads, 0, h.stream2>>>(P, h.y.p, h.st.p);
        k_primal_panels_chk<<<(unsigned)ceil_div(h.PT.R, kBlock), kBlock, 0, h.stream2>>>(
            P, h.x.p, h.c.p, h.lv.p, h.uv.p, h.xhat.p, h.xext.p, h.aty.p, h.st.p, tau_override);
        PDHG_HIP(hipEventRecord(h.ev_join, h.stream2));
        const int32_t ns = h.AT.nslices - h.sell_skip;
        if (ns > 0)
            k_primal_sell_chk<<<(unsigned)ceil_div(ns, kBlock / 64), kBlock, 0, h.stream>>>(
                view(h.AT), h.sell_skip, h.y.p, h.x.p, h.c.p, h.lv.p, h.uv.p, h.xhat.p, h.xext.p,
                h.aty.p, h.st.p, tau_override);
        PDHG_HIP(hipStreamWaitEvent(h.stream, h.ev_join, 0));
        return;
    }
    k_primal_chk<<<grid_of(h.AT), kBlock, 0, h.stream>>>(
        view(h.AT), h.y.p, h.x.p, h.c.p, h.lv.p, h.uv.p,
        h.xhat.p, h.xext.p, h.aty.p, h.st.p, tau_override);
}

void launch_dual_check(Handle &h, double sigma_override) {
    if (h.dense) {
        dense_dual_check(h, sigma_override);
        return;
    }
    if (h.A.nblocks() == 0) return;
    k_dual_chk<<<grid_of(h.A), kBlock, 0, h.stream>>>(view(h.A), h.xext.p, h.y.p, h.lc.p,
                                                      h.uc.p, h.yhat.p, h.st.p, sigma_override);
}

// Blocks of column-side check partials that launch_check_sums writes.
int32_t check_n_blocks(const Handle &h) {
    if (h.PT.R == 0) return h.AT.nblocks();
    const int32_t ns = h.AT.nslices - h.sell_skip;
    return (ns > 0 ? (int32_t)ceil_div(ns, kBlock / 64) : 0) + (int32_t)ceil_div(h.PT.R, kBlock);
}

void launch_check_sums(Handle &h) {
    if (h.dense) {
        dense_check_sums(h);
        return;
    }
    if (h.AT.nblocks() && h.PT.R > 0) {
        // as launch_primal: the panel rows on stream2 beside the SELL-64 rest;
        // block partials [0, sell blocks) from the rest, then the panel rows'
        const PanelView P = view(h.PT);
        const int32_t ns = h.AT.nslices - h.sell_skip;
        const int32_t sell_blocks = ns > 0 ? (int32_t)ceil_div(ns, kBlock / 64) : 0;
        PDHG_HIP(hipEventRecord(h.ev_fork, h.stream));
        PDHG_HIP(hipStreamWaitEvent(h.stream2, h.ev_fork, 0));
        k_panel_dot<<<h.PT.nwg, kPanelThreads, 0, h.stream2>>>(P, h.yhat.p, h.st.p);
        k_check_n_panels<<<(unsigned)ceil_div(h.PT.R, kBlock), kBlock, 0, h.stream2>>>(
            P, sell_blocks, h.xhat.p, h.x.p, h.x0.p, h.aty.p, h.Dc.p, h.c_o.p, h.lv_o.p, h.uv_o.p,
            h.pn.p, h.q0.p, h.qhat.p, h.prn.p, h.st.p);
        PDHG_HIP(hipEventRecord(h.ev_join, h.stream2));
        if (sell_blocks > 0)
            k_check_n_sell<<<(unsigned)sell_blocks, kBlock, 0, h.stream>>>(
                view(h.AT), h.sell_skip, h.yhat.p, h.xhat.p, h.x.p, h.x0.p, h.aty.p, h.Dc.p,
                h.c_o.p, h.lv_o.p, h.uv_o.p, h.pn.p, h.q0.p, h.qhat.p, h.prn.p, h.st.p);
        PDHG_HIP(hipStreamWaitEvent(h.stream, h.ev_join, 0));
    } else if (h.AT.nblocks()) {
        k_check_n<<<grid_of(h.AT), kBlock, 0, h.stream>>>(
            view(h.AT), h.yhat.p, h.xhat.p, h.x.p,
            h.x0.p, h.aty.p, h.Dc.p, h.c_o.p, h.lv_o.p, h.uv_o.p, h.pn.p, h.q0.p, h.qhat.p,
            h.prn.p, h.st.p);
    }
    if (h.A.nblocks())
        k_check_m<<<grid_of(h.A), kBlock, 0, h.stream>>>(
            view(h.A), h.xhat.p, h.yhat.p, h.y.p, h.y0.p,
            h.Dr.p, h.lc_o.p, h.uc_o.p, h.pm.p, h.p0.p, h.phat.p, h.prm.p, h.st.p);
}

void launch_controller(Handle &h, int32_t chunk_plain, int32_t is_last, int32_t last_status) {
    CtlConst K;
    K.eps = h.polish ? h.opt.eps_feas_polish : h.opt.eps;
    K.bnorm = h.bnorm;
    K.cnorm = h.cnorm;
    K.eta = h.eta;
    K.beta_suff = h.opt.restart_sufficient;
    K.beta_nec = h.opt.restart_necessary;
    K.beta_art = h.opt.restart_artificial;
    K.qp = 0;
    K.detect = !h.polish && (h.opt.eps_primal_infeasible > 0.0 || h.opt.eps_dual_infeasible > 0.0);
    K.eps_pinf = h.opt.eps_primal_infeasible;
    K.eps_dinf = h.opt.eps_dual_infeasible;
    K.term = h.polish;
    K.pad = 0;
    k_controller<<<1, kBlock, 0, h.stream>>>(h.st.p, h.pn.p, h.nbn, h.pm.p, h.nbm, h.prn.p,
                                              h.prm.p, K, chunk_plain, is_last, last_status);
}

void launch_apply(Handle &h) {
    const int64_t tot = (int64_t)h.n + h.m;
    k_apply<<<(unsigned)ceil_div(tot, kBlock), kBlock, 0, h.stream>>>(
        h.st.p, h.n, h.m, h.x.p, h.x0.p, h.xhat.p, h.y.p, h.y0.p, h.yhat.p, h.opt.gamma,
        h.q0.p, h.qhat.p, h.p0.p, h.phat.p);
}

// On an infeasibility certificate the finalised output carries the ray:
// xhat <- (xhat - x0) s (primal ray) or yhat <- (yhat - y0) s (dual ray),
// s = st->ray_scale; the finalize then applies D_c / D_r. A QP's finalised
// points are the averages xbar / ybar.
__global__ __launch_bounds__(kBlock) void k_make_ray(const DevState *__restrict__ st, int32_t len,
                                                     double *__restrict__ v,
                                                     const double *__restrict__ v0) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) v[i] = (v[i] - v0[i]) * st->ray_scale;
}

// Finite entries of a bound vector set to 0 (the dual polishing problem).
__global__ __launch_bounds__(kBlock) void k_zero_finite(int32_t len, double *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len && isfinite(v[i])) v[i] = 0.0;
}

void launch_zero_finite(Handle &h, double *v, int32_t len) {
    if (len <= 0) return;
    k_zero_finite<<<(unsigned)ceil_div(len, kBlock), kBlock, 0, h.stream>>>(len, v);
    PDHG_HIP(hipGetLastError());
}

void launch_make_ray(Handle &h, int32_t status) {
    double *xv = h.q_kind ? h.xbar.p : h.xhat.p, *yv = h.q_kind ? h.ybar.p : h.yhat.p;
    if (status == PDHG_PRIMAL_INFEASIBLE && h.m > 0)
        k_make_ray<<<(unsigned)ceil_div(h.m, kBlock), kBlock, 0, h.stream>>>(h.st.p, h.m, yv, h.y0.p);
    if (status == PDHG_DUAL_INFEASIBLE && h.n > 0)
        k_make_ray<<<(unsigned)ceil_div(h.n, kBlock), kBlock, 0, h.stream>>>(h.st.p, h.n, xv, h.x0.p);
    PDHG_HIP(hipGetLastError());
}

void launch_debug_halpern(Handle &h, int64_t k, double *xnew_int, double *ynew_int) {
    const int64_t tot = (int64_t)h.n + h.m;
    k_halpern_explicit<<<(unsigned)ceil_div(tot, kBlock), kBlock, 0, h.stream>>>(
        h.n, h.m, k, h.x.p, h.x0.p, h.xhat.p, h.y.p, h.y0.p, h.yhat.p, xnew_int, ynew_int,
        h.opt.gamma);
}

void launch_init_point(Handle &h, const double *x_init, const double *y_init) {
    const int64_t tot = (int64_t)h.n + h.m;
    k_init_point<<<(unsigned)ceil_div(tot, kBlock), kBlock, 0, h.stream>>>(
        h.n, h.m, h.perm_c.p, h.perm_r.p, x_init, y_init, h.Dc.p, h.Dr.p, h.lv.p, h.uv.p, h.lc.p,
        h.uc.p, h.x.p, h.x0.p, h.y.p, h.y0.p);
}

void launch_finalize(Handle &h, double *x_out, double *y_out) {
    if (h.n) launch_scatter_scaled(h.stream, h.perm_c.p, h.Dc.p, h.xhat.p, x_out, h.n);
    if (h.m) launch_scatter_scaled(h.stream, h.perm_r.p, h.Dr.p, h.yhat.p, y_out, h.m);
}

void launch_reset_state(Handle &h) {
    k_reset_state<<<1, 64, 0, h.stream>>>(h.st.p, h.eta, h.omega0);
}

void launch_gather(hipStream_t s, const int32_t *perm, const double *src, double *dst,
                   int32_t len) {
    if (len <= 0) return;
    k_gather<<<(unsigned)ceil_div(len, kBlock), kBlock, 0, s>>>(perm, src, dst, len);
}

void launch_scatter(hipStream_t s, const int32_t *perm, const double *src, double *dst,
                    int32_t len) {
    if (len <= 0) return;
    k_scatter<<<(unsigned)ceil_div(len, kBlock), kBlock, 0, s>>>(perm, src, dst, len);
}

void launch_scatter_scaled(hipStream_t s, const int32_t *perm, const double *scale,
                           const double *src, double *dst, int32_t len) {
    if (len <= 0) return;
    k_scatter_scaled<<<(unsigned)ceil_div(len, kBlock), kBlock, 0, s>>>(perm, scale, src, dst,
                                                                        len);
}

}  // namespace pdhg
