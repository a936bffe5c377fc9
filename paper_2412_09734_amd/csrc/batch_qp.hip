// Batched rAPDHG (Algorithm 2) for QPs with a shared constraint matrix and
// Q_b = F F' + diag(d_b): F (n x r) shared by the batch, d_b per instance.
// One workgroup per instance, as in batch.hip. The scaling depends on A only,
// so F~ = D_c F is shared and d~_b = D_c^2 d_b. Per iteration and instance:
//   v = (1-beta) xbar + beta x;  t = F~' v (workgroup tree);  qv = F~ t + d~ v
//   x+ = clamp(x - tau_k (qv + c - A~'y)), xext = 2 x+ - x, xbar update
//   y+ = dual prox with A~ xext, ybar update
// Checks on the averages with the weighted KKT restart metric. The unrolled
// variant records the schedule and projection states and keeps the state
// every kCkpt iterations; the reverse pass recomputes each segment from its
// checkpoint (the momentum points v are needed for the gradient in d).
#include <algorithm>
#include <memory>
#include <vector>

#include "device.hpp"

namespace pdhg {

constexpr int kRmax = 32;   // largest supported rank of F
constexpr int kCkpt = 50;   // checkpoint spacing of the unrolled QP
constexpr int kWaveRowsMax = 256;   // row limit of the wave-per-row mode

struct QArgs {
    int32_t B, m, n, r;
    int32_t wave_rows;      // 1: each constraint row is reduced by one wave (few, long rows)
    const int32_t *arp, *aci, *trp, *tci;
    const double *ava, *tva, *Dr, *Dc;
    double eta;
    const double *FT;       // F~' [r_pad][n], r_pad = r rounded up to 8, zero rows past r
    const double *d_o;      // original d [B][n]
    double *normq;          // [B]
    const double *c_o, *lc_o, *uc_o, *lv_o, *uv_o;
    double *c, *lc, *uc, *lv, *uv, *dd;   // scaled, per instance
    double *x, *y, *xb, *yb, *x0, *y0, *xe, *v;
    const double *x_init, *y_init;
    double *x_out, *y_out;
    double *res;            // [B][12]
    int32_t *queue;
    // unrolled
    int64_t T;
    int32_t replay;
    uint8_t *restart;
    double *omega;
    int32_t *kk;
    uint64_t *xmask, *ymask;   // [B][T][words]
    double *ckpt;              // [B][nck][2n + 2m]
    double *vseg;              // [B][kCkpt][n]
    double *vall;              // [B][T][n] every momentum point, or null (recompute from checkpoints)
    const double *gx, *gy;
    double *gc, *glc, *guc, *gd;
    double *bxb, *byb, *bw, *bqv;   // reverse scratch
};

struct QOpts {
    double eps, gamma, beta_suff, beta_nec, beta_art, power_tol;
    double eps_pinf, eps_dinf;   // infeasibility certificate tolerances
    int64_t limit;
    int32_t check_every, power_max_iters;
    int32_t detect, pad;         // 1: test the rays at checks
};

template <int BT, int K>
__device__ __forceinline__ void qsum(double (&v)[K]) {
    constexpr int NW = BT / 64;
    __shared__ double sh[K][NW];
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
        for (int w = 0; w < NW; ++w) s += sh[q][w];
        v[q] = s;
    }
    __syncthreads();
}

template <int BT>
__device__ __forceinline__ int32_t qnext(int32_t *queue) {
    __shared__ int32_t id;
    if (threadIdx.x == 0) id = atomicAdd(queue, 1);
    __syncthreads();
    const int32_t r = id;
    __syncthreads();
    return r;
}

__device__ __forceinline__ double qdot(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                       const double *__restrict__ va, int32_t row,
                                       const double *__restrict__ v) {
    double acc = 0.0;
    for (int32_t e = rp[row]; e < rp[row + 1]; ++e) acc = fma(va[e], v[ci[e]], acc);
    return acc;
}

// Row dot by one wave: lanes stride over the row, butterfly sum (all lanes).
__device__ __forceinline__ double qdot_wave(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                            const double *__restrict__ va, int32_t row,
                                            const double *__restrict__ v) {
    double acc = 0.0;
    for (int32_t e = rp[row] + (int32_t)(threadIdx.x & 63); e < rp[row + 1]; e += 64)
        acc = fma(va[e], v[ci[e]], acc);
    return wave_sum(acc);
}

// Per-instance pointers.
struct QI {
    double *c, *lc, *uc, *lv, *uv, *dd, *x, *y, *xb, *yb, *x0, *y0, *xe, *v;
    const double *c_o, *lc_o, *uc_o, *lv_o, *uv_o, *d_o;
};

__device__ __forceinline__ QI qinst(const QArgs &a, int32_t b) {
    const size_t vn = (size_t)b * a.n, vm = (size_t)b * a.m;
    QI q;
    q.c = a.c + vn; q.lv = a.lv + vn; q.uv = a.uv + vn; q.dd = a.dd + vn;
    q.x = a.x + vn; q.xb = a.xb + vn; q.x0 = a.x0 + vn; q.xe = a.xe + vn; q.v = a.v + vn;
    q.lc = a.lc + vm; q.uc = a.uc + vm; q.y = a.y + vm; q.yb = a.yb + vm; q.y0 = a.y0 + vm;
    q.c_o = a.c_o + vn; q.lv_o = a.lv_o + vn; q.uv_o = a.uv_o + vn; q.d_o = a.d_o + vn;
    q.lc_o = a.lc_o + vm; q.uc_o = a.uc_o + vm;
    return q;
}

// On-chip variant: the instance's scaled data and iterates in dynamic LDS
// (9 n-vectors c~, l~_v, u~_v, d~, x, xbar, x0, x_ext, v and 5 m-vectors
// l~_c, u~_c, y, ybar, y0). Every one of them is written before it is read
// (scaling, initial point, or within the step), so nothing is copied in.
constexpr size_t kQOnchipBytes = 56 * 1024;

__host__ __device__ inline size_t q_onchip_bytes(int32_t n, int32_t m) {
    return (9 * (size_t)n + 5 * (size_t)m) * sizeof(double);
}

// The reverse pass adds its cotangent scratch (2 n- and 2 m-vectors).
__host__ __device__ inline size_t q_onchip_bytes_bwd(int32_t n, int32_t m) {
    return (11 * (size_t)n + 7 * (size_t)m) * sizeof(double);
}

__device__ __forceinline__ void q_onchip(const QArgs &a, QI &q, double *lds) {
    double *p = lds;
    q.c = p; p += a.n;
    q.lv = p; p += a.n;
    q.uv = p; p += a.n;
    q.dd = p; p += a.n;
    q.x = p; p += a.n;
    q.xb = p; p += a.n;
    q.x0 = p; p += a.n;
    q.xe = p; p += a.n;
    q.v = p; p += a.n;
    q.lc = p; p += a.m;
    q.uc = p; p += a.m;
    q.y = p; p += a.m;
    q.yb = p; p += a.m;
    q.y0 = p;
}

// (Q~ v)_j = (F~ t)_j + d~_j v_j with t = F~'v from qt_of (in LDS)
__device__ __forceinline__ double qv_row(const QArgs &a, const QI &q, int32_t j, const double *t,
                                         const double *vv) {
    constexpr int U = 4;   // independent loads in flight; the sum stays in order of p
    const double *__restrict__ fj = a.FT + j;
    const size_t n = (size_t)a.n;
    double acc = 0.0;
    int32_t p = 0;
    for (; p + U <= a.r; p += U) {
        double f[U];
#pragma unroll
        for (int u = 0; u < U; ++u) f[u] = fj[(size_t)(p + u) * n];
#pragma unroll
        for (int u = 0; u < U; ++u) acc = fma(f[u], t[p + u], acc);
    }
    for (; p < a.r; ++p) acc = fma(fj[(size_t)p * n], t[p], acc);
    return acc + q.dd[j] * vv[j];
}

// Eight wave sums at once: the first three butterfly steps (lane bits 5, 4, 3)
// each halve the values a lane carries, so 3 + 3 + 1 exchanges of the last
// value finish the job instead of 8 x 6. Lane l ends with the total of
// value 4 bit3(l) + 2 bit4(l) + bit5(l).
__device__ __forceinline__ double wave_sum_x8(const double (&s)[8]) {
    const int lane = (int)(threadIdx.x & 63);
    double a[4], b[2];
    const bool h5 = (lane >> 5) & 1, h4 = (lane >> 4) & 1, h3 = (lane >> 3) & 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double keep = h5 ? s[2 * i + 1] : s[2 * i];
        const double send = h5 ? s[2 * i] : s[2 * i + 1];
        a[i] = keep + __shfl_xor(send, 32);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double keep = h4 ? a[2 * i + 1] : a[2 * i];
        const double send = h4 ? a[2 * i] : a[2 * i + 1];
        b[i] = keep + __shfl_xor(send, 16);
    }
    double c = (h3 ? b[1] : b[0]) + __shfl_xor(h3 ? b[0] : b[1], 8);
    c += __shfl_xor(c, 4);
    c += __shfl_xor(c, 2);
    c += __shfl_xor(c, 1);
    return c;
}

// t = F~' w over the instance: per p, each thread's columns in order, then the
// wave reduction and the waves in order (eight values of p per pass). The r values land in LDS, where every
// thread reads them (a register array indexed by the runtime rank would live
// in scratch memory). The next call overwrites them.
template <int BT>
__device__ __forceinline__ const double *qt_of(const QArgs &a, const double *w) {
    constexpr int NW = BT / 64;
    __shared__ double sh[kRmax][NW];
    __shared__ double t[kRmax];
    constexpr int U = 8;   // factor columns per pass (wave_sum_x8)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t n = (size_t)a.n;
    for (int32_t p0 = 0; p0 < a.r; p0 += U) {
        const double *__restrict__ fp = a.FT + (size_t)p0 * n;
        double s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) s[u] = 0.0;
        // F~' has zero rows up to a multiple of 8: the loads need no guard
        for (int32_t j = threadIdx.x; j < a.n; j += BT) {
            const double wj = w[j];
#pragma unroll
            for (int u = 0; u < U; ++u) s[u] = fma(fp[(size_t)u * n + j], wj, s[u]);
        }
        const double ws = wave_sum_x8(s);
        const int u = 4 * ((lane >> 3) & 1) + 2 * ((lane >> 4) & 1) + ((lane >> 5) & 1);
        if ((lane & 7) == 0 && p0 + u < a.r) sh[p0 + u][wave] = ws;
    }
    __syncthreads();
    if ((int32_t)threadIdx.x < a.r) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) s += sh[threadIdx.x][v];
        t[threadIdx.x] = s;
    }
    __syncthreads();
    return t;
}

// Transformed data and the norms of one instance.
template <int BT>
__device__ __forceinline__ void qprepare(const QArgs &a, const QI &q, double &cn, double &bn,
                                         double &cnorm, double &bnorm) {
    double nrm[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t j = threadIdx.x; j < a.n; j += BT) {
        const double d = a.Dc[j];
        const double cj = d * q.c_o[j];
        q.c[j] = cj;
        q.lv[j] = q.lv_o[j] / d;
        q.uv[j] = q.uv_o[j] / d;
        q.dd[j] = (d * d) * q.d_o[j];
        nrm[0] += cj * cj;
        nrm[2] += q.c_o[j] * q.c_o[j];
    }
    for (int32_t i = threadIdx.x; i < a.m; i += BT) {
        const double d = a.Dr[i];
        const double l = d * q.lc_o[i], u = d * q.uc_o[i];
        q.lc[i] = l;
        q.uc[i] = u;
        double bb = 0.0, bo = 0.0;
        if (isfinite(l)) bb = fmax(bb, fabs(l));
        if (isfinite(u)) bb = fmax(bb, fabs(u));
        if (isfinite(q.lc_o[i])) bo = fmax(bo, fabs(q.lc_o[i]));
        if (isfinite(q.uc_o[i])) bo = fmax(bo, fabs(q.uc_o[i]));
        nrm[1] += bb * bb;
        nrm[3] += bo * bo;
    }
    qsum<BT, 4>(nrm);
    cn = sqrt(nrm[0]);
    bn = sqrt(nrm[1]);
    cnorm = sqrt(nrm[2]);
    bnorm = sqrt(nrm[3]);
}

template <int BT>
__device__ __forceinline__ void qinit(const QArgs &a, const QI &q, const double *xi, const double *yi) {
    for (int32_t j = threadIdx.x; j < a.n; j += BT) {
        const double v0 = xi ? xi[j] / a.Dc[j] : 0.0;
        const double xv = clampd(v0, q.lv[j], q.uv[j]);
        q.x[j] = xv;
        q.x0[j] = xv;
        q.xb[j] = xv;
    }
    for (int32_t i = threadIdx.x; i < a.m; i += BT) {
        const double v0 = yi ? yi[i] / a.Dr[i] : 0.0;
        const double lo = isfinite(q.uc[i]) ? -INFINITY : 0.0;
        const double hi = isfinite(q.lc[i]) ? INFINITY : 0.0;
        const double yv = clampd(v0, lo, hi);
        q.y[i] = yv;
        q.y0[i] = yv;
        q.yb[i] = yv;
    }
    __syncthreads();
}

// One rAPDHG iteration; optionally records the projection states.
template <int BT>
__device__ __forceinline__ void qstep(const QArgs &a, const QI &q, int64_t k, double omega,
                                      double normq, uint64_t *xmt, uint64_t *ymt) {
    const double beta = 2.0 / (double)(k + 2), theta = beta;
    const double tau = 1.0 / (omega / a.eta + 2.0 * normq / (double)(k + 1));
    const double sigma = a.eta * omega;
    for (int32_t j = threadIdx.x; j < a.n; j += BT) q.v[j] = (1.0 - beta) * q.xb[j] + beta * q.x[j];
    const double *t = qt_of<BT>(a, q.v);
    for (int32_t j0 = 0; j0 < a.n; j0 += BT) {
        const int32_t j = j0 + (int32_t)threadIdx.x;
        bool inside = false;
        if (j < a.n) {
            const double qv = qv_row(a, q, j, t, q.v);
            const double s = qdot(a.trp, a.tci, a.tva, j, q.y);
            const double xr = q.x[j];
            const double u = xr - tau * (qv + q.c[j] - s);
            inside = u > q.lv[j] && u < q.uv[j];
            const double xp = clampd(u, q.lv[j], q.uv[j]);
            q.xe[j] = 2.0 * xp - xr;
            q.x[j] = xp;
            q.xb[j] = (1.0 - theta) * q.xb[j] + theta * xp;
        }
        if (xmt) {
            const uint64_t bits = __ballot(inside);
            if ((threadIdx.x & 63) == 0 && j < a.n) xmt[j >> 6] = bits;
        }
    }
    __syncthreads();
    if (a.wave_rows) {
        // few long rows: one wave per row, projection states staged in LDS
        __shared__ uint8_t flags[kWaveRowsMax];
        for (int32_t i = (int32_t)(threadIdx.x >> 6); i < a.m; i += BT / 64) {
            const double av = qdot_wave(a.arp, a.aci, a.ava, i, q.xe);
            if ((threadIdx.x & 63) == 0) {
                const double w = q.y[i] / sigma - av;
                const bool at_u = w < -q.uc[i], at_l = w > -q.lc[i];
                const double yp = sigma * (w - clampd(w, -q.uc[i], -q.lc[i]));
                q.y[i] = yp;
                q.yb[i] = (1.0 - theta) * q.yb[i] + theta * yp;
                flags[i] = (uint8_t)((at_u ? 1 : 0) | (at_l ? 2 : 0));
            }
        }
        __syncthreads();
        if (ymt) {
            for (int32_t i0 = 0; i0 < a.m; i0 += BT) {
                const int32_t i = i0 + (int32_t)threadIdx.x;
                const uint8_t fl = i < a.m ? flags[i] : (uint8_t)0;
                const uint64_t bu = __ballot((fl & 1) != 0), bl = __ballot((fl & 2) != 0);
                if ((threadIdx.x & 63) == 0 && i < a.m) {
                    ymt[2 * (i >> 6)] = bu;
                    ymt[2 * (i >> 6) + 1] = bl;
                }
            }
        }
        __syncthreads();
        return;
    }
    for (int32_t i0 = 0; i0 < a.m; i0 += BT) {
        const int32_t i = i0 + (int32_t)threadIdx.x;
        bool at_u = false, at_l = false;
        if (i < a.m) {
            const double av = qdot(a.arp, a.aci, a.ava, i, q.xe);
            const double w = q.y[i] / sigma - av;
            at_u = w < -q.uc[i];
            at_l = w > -q.lc[i];
            const double yp = sigma * (w - clampd(w, -q.uc[i], -q.lc[i]));
            q.y[i] = yp;
            q.yb[i] = (1.0 - theta) * q.yb[i] + theta * yp;
        }
        if (ymt) {
            const uint64_t bu = __ballot(at_u), bl = __ballot(at_l);
            if ((threadIdx.x & 63) == 0 && i < a.m) {
                ymt[2 * (i >> 6)] = bu;
                ymt[2 * (i >> 6) + 1] = bl;
            }
        }
    }
    __syncthreads();
}

// KKT terms of the averages in the original space:
//  0 |xbar-x0|^2 1 |r_d|^2 2 x'Qx 3 c'x 4 l_v'lam+ - u_v'lam- 5 |r_p|^2 6 l_c'y+ - u_c'y- 7 |ybar-y0|^2
template <int BT>
__device__ __forceinline__ void qcheck(const QArgs &a, const QI &q, double (&v)[8]) {
    const double *t = qt_of<BT>(a, q.xb);
#pragma unroll
    for (int p = 0; p < 8; ++p) v[p] = 0.0;
    for (int32_t j = threadIdx.x; j < a.n; j += BT) {
        const double xb = q.xb[j];
        const double d0 = xb - q.x0[j];
        v[0] += d0 * d0;
        const double qx = qv_row(a, q, j, t, q.xb) / a.Dc[j];
        const double s = qdot(a.trp, a.tci, a.tva, j, q.yb);
        const double d = a.Dc[j];
        const double xo = d * xb;
        const double g = qx + q.c_o[j] - s / d;
        const double lo = q.lv_o[j], hi = q.uv_o[j];
        const bool lf = isfinite(lo), uf = isfinite(hi);
        const double lam = (!lf && !uf) ? 0.0 : (lf && !uf) ? fmax(g, 0.0) : (!lf && uf) ? fmin(g, 0.0) : g;
        const double rd = g - lam;
        v[1] += rd * rd;
        v[2] += xo * qx;
        v[3] += q.c_o[j] * xo;
        v[4] += (lf ? lo * fmax(lam, 0.0) : 0.0) - (uf ? hi * fmax(-lam, 0.0) : 0.0);
    }
    const bool wr = a.wave_rows != 0;
    for (int32_t i = wr ? (int32_t)(threadIdx.x >> 6) : (int32_t)threadIdx.x; i < a.m;
         i += wr ? BT / 64 : BT) {
        const double p = wr ? qdot_wave(a.arp, a.aci, a.ava, i, q.xb) : qdot(a.arp, a.aci, a.ava, i, q.xb);
        if (wr && (threadIdx.x & 63) != 0) continue;
        const double d = a.Dr[i];
        const double ax = p / d;
        const double lo = q.lc_o[i], hi = q.uc_o[i];
        const double rpr = ax - clampd(ax, lo, hi);
        v[5] += rpr * rpr;
        const double yb = q.yb[i];
        const double yo = d * yb;
        v[6] += (isfinite(lo) ? lo * fmax(yo, 0.0) : 0.0) - (isfinite(hi) ? hi * fmax(-yo, 0.0) : 0.0);
        const double d0 = yb - q.y0[i];
        v[7] += d0 * d0;
    }
    qsum<BT, 8>(v);
}

template <int BT, int K>
__device__ __forceinline__ void qmax(double (&v)[K]) {
    constexpr int NW = BT / 64;
    __shared__ double sh[K][NW];
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
        for (int w = 1; w < NW; ++w) s = fmax(s, sh[q][w]);
        v[q] = s;
    }
    __syncthreads();
}

// Ray terms of the averages against the restart anchor (the certificates of
// Section 3's infeasibility detection): dx = D_c (xbar - x0), dy = D_r (ybar - y0)
// in the original space. The scaled difference xbar - x0 goes to q.v (free
// between iterations). rs: 0 dual-ray objective (columns), 1 c'dx, 2 dual-ray
// objective (rows); rm: 0 dual-ray violation, 1 primal-ray violation including
// |Q dx|.
template <int BT>
__device__ __forceinline__ void qray(const QArgs &a, const QI &q, double (&rs)[3], double (&rm)[2]) {
    for (int32_t j = threadIdx.x; j < a.n; j += BT) q.v[j] = q.xb[j] - q.x0[j];
    rs[0] = rs[1] = rs[2] = 0.0;
    rm[0] = rm[1] = 0.0;
    {
        // |Q dx| first: F~'(xbar - x0) is live in this loop only
        const double *t = qt_of<BT>(a, q.v);
        for (int32_t j = threadIdx.x; j < a.n; j += BT) rm[1] = fmax(rm[1], fabs(qv_row(a, q, j, t, q.v) / a.Dc[j]));
    }
    for (int32_t j = threadIdx.x; j < a.n; j += BT) {
        const double d = a.Dc[j];
        const double sh = qdot(a.trp, a.tci, a.tva, j, q.yb);
        const double s0 = qdot(a.trp, a.tci, a.tva, j, q.y0);
        double s[2], mx[2];
        ray_col_terms(sh, s0, d, q.v[j], q.c_o[j], q.lv_o[j], q.uv_o[j], s, mx);
        rs[0] += s[0];
        rs[1] += s[1];
        rm[0] = fmax(rm[0], mx[0]);
        rm[1] = fmax(rm[1], mx[1]);
    }
    const bool wr = a.wave_rows != 0;
    for (int32_t i = wr ? (int32_t)(threadIdx.x >> 6) : (int32_t)threadIdx.x; i < a.m;
         i += wr ? BT / 64 : BT) {
        const double p = wr ? qdot_wave(a.arp, a.aci, a.ava, i, q.v) : qdot(a.arp, a.aci, a.ava, i, q.v);
        if (wr && (threadIdx.x & 63) != 0) continue;
        double s[1], mx[2];
        ray_row_terms(p, 0.0, a.Dr[i], q.yb[i] - q.y0[i], q.lc_o[i], q.uc_o[i], s, mx);
        rs[2] += s[0];
        rm[0] = fmax(rm[0], mx[0]);
        rm[1] = fmax(rm[1], mx[1]);
    }
    qsum<BT, 3>(rs);
    qmax<BT, 2>(rm);
}

template <int BT>
__device__ __forceinline__ void qrestart(const QArgs &a, const QI &q) {
    for (int32_t j = threadIdx.x; j < a.n; j += BT) {
        q.x[j] = q.xb[j];
        q.x0[j] = q.xb[j];
    }
    for (int32_t i = threadIdx.x; i < a.m; i += BT) {
        q.y[i] = q.yb[i];
        q.y0[i] = q.yb[i];
    }
    __syncthreads();
}

// ||Q~_b||_2 per instance: power iteration with the Rayleigh quotient.
template <int BT>
__global__ __launch_bounds__(BT) void k_bqp_norm(QArgs a, QOpts o) {
    for (;;) {
        const int32_t b = qnext<BT>(a.queue);
        if (b >= a.B) return;
        const QI q = qinst(a, b);
        for (int32_t j = threadIdx.x; j < a.n; j += BT) {
            const double d = a.Dc[j];
            q.dd[j] = (d * d) * q.d_o[j];
        }
        double *vv = q.xe, *ww = q.v;
        double s1[1] = {0.0};
        for (int32_t j = threadIdx.x; j < a.n; j += BT) {
            uint64_t z = (uint64_t)j + 0x9e3779b97f4a7c15ull;
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
            z = z ^ (z >> 31);
            const double val = 0.5 + (double)(z >> 11) * 0x1.0p-53;
            vv[j] = val;
            s1[0] += val * val;
        }
        qsum<BT, 1>(s1);
        const double nv = sqrt(s1[0]);
        for (int32_t j = threadIdx.x; j < a.n; j += BT) vv[j] = vv[j] / nv;
        __syncthreads();
        double lam = 0.0, lam_prev = 0.0;
        for (int32_t it = 1; it <= o.power_max_iters; ++it) {
            const double *t = qt_of<BT>(a, vv);
            double s2[2] = {0.0, 0.0};
            for (int32_t j = threadIdx.x; j < a.n; j += BT) {
                const double w = qv_row(a, q, j, t, vv);
                ww[j] = w;
                s2[0] += vv[j] * w;
                s2[1] += w * w;
            }
            qsum<BT, 2>(s2);
            lam = s2[0];
            const double nw = sqrt(s2[1]);
            if (!(nw > 0.0)) {
                lam = 0.0;
                break;
            }
            for (int32_t j = threadIdx.x; j < a.n; j += BT) vv[j] = ww[j] / nw;
            __syncthreads();
            if (it > 1 && fabs(lam - lam_prev) <= o.power_tol * fabs(lam)) break;
            lam_prev = lam;
        }
        if (threadIdx.x == 0) a.normq[b] = lam;
        __syncthreads();
    }
}

template <int BT, bool RAYS, bool ONCHIP>
__global__ __launch_bounds__(BT) void k_bqp_solve(QArgs a, QOpts o) {
    extern __shared__ double qlds[];
    for (;;) {
        const int32_t b = qnext<BT>(a.queue);
        if (b >= a.B) return;
        QI q = qinst(a, b);
        if (ONCHIP) q_onchip(a, q, qlds);
        double cn, bn, cnorm, bnorm;
        qprepare<BT>(a, q, cn, bn, cnorm, bnorm);
        qinit<BT>(a, q, a.x_init ? a.x_init + (size_t)b * a.n : nullptr,
                  a.y_init ? a.y_init + (size_t)b * a.m : nullptr);
        const double normq = a.normq[b];
        double omega = (cn > 1e-10 && bn > 1e-10) ? cn / bn : 1.0;
        int64_t t = 0, k = 0, restarts = 0;
        double r_start = 0.0, r_prev = 0.0, P = 0.0, D = 0.0, kkt = 0.0, rp = 0.0, rd = 0.0, rg = 0.0;
        int32_t status = 0;
        double ray_scale = 0.0;
        for (;;) {
            qstep<BT>(a, q, k, omega, normq, nullptr, nullptr);
            const bool check = (t % o.check_every) == 0;
            const bool last = t + 1 >= o.limit;
            if (check || last) {
                double v[8];
                qcheck<BT>(a, q, v);
                P = 0.5 * v[2] + v[3];
                D = -0.5 * v[2] + v[6] + v[4];
                const double ap = sqrt(v[5]), ad = sqrt(v[1]), ag = fabs(P - D);
                rp = ap / (1.0 + bnorm);
                rd = ad / (1.0 + cnorm);
                rg = ag / (1.0 + fabs(P) + fabs(D));
                kkt = rp;
                if (rd > kkt || isnan(rd)) kkt = rd;
                if (rg > kkt || isnan(rg)) kkt = rg;
                if (isnan(kkt)) { status = PDHG_NUMERICAL_ERROR; break; }
                if (kkt <= o.eps) { status = PDHG_OPTIMAL; break; }
                // the anchor is a restart point once a restart has happened
                if (RAYS && restarts > 0) {
                    double rs[3], rm[2];
                    qray<BT>(a, q, rs, rm);
                    const double obj_d = rs[0] + rs[2], obj_p = rs[1];
                    if (o.eps_pinf > 0.0 && obj_d > 0.0 && rm[0] <= o.eps_pinf * obj_d) {
                        status = PDHG_PRIMAL_INFEASIBLE;
                        ray_scale = 1.0 / obj_d;
                        break;
                    }
                    if (o.eps_dinf > 0.0 && obj_p < 0.0 && rm[1] <= o.eps_dinf * (-obj_p)) {
                        status = PDHG_DUAL_INFEASIBLE;
                        ray_scale = -1.0 / obj_p;
                        break;
                    }
                }
                if (last) { status = PDHG_ITERATION_LIMIT; break; }
                const double r = sqrt(omega * ap * ap + ad * ad / omega + ag * ag);
                bool restart = false;
                if (t == 0) {
                    r_start = r;
                    r_prev = r;
                } else if (r <= o.beta_suff * r_start || (r <= o.beta_nec * r_start && r > r_prev) ||
                           (double)k >= o.beta_art * (double)t) {
                    restart = true;
                } else {
                    r_prev = r;
                }
                if (restart) {
                    const double dxr = sqrt(v[0]), dyr = sqrt(v[7]);
                    omega = batch_new_omega(omega, dxr, dyr);
                    qrestart<BT>(a, q);
                    k = 0;
                    r_start = r;
                    r_prev = r;
                    ++restarts;
                } else {
                    ++k;
                }
            } else {
                ++k;
            }
            ++t;
        }
        // a certificate replaces the average it was found from, scaled to
        // objective 1 (dual ray) or -1 (primal ray)
        const bool xray = status == PDHG_DUAL_INFEASIBLE, yray = status == PDHG_PRIMAL_INFEASIBLE;
        for (int32_t j = threadIdx.x; j < a.n; j += BT)
            a.x_out[(size_t)b * a.n + j] = a.Dc[j] * (xray ? (q.xb[j] - q.x0[j]) * ray_scale : q.xb[j]);
        for (int32_t i = threadIdx.x; i < a.m; i += BT)
            a.y_out[(size_t)b * a.m + i] = a.Dr[i] * (yray ? (q.yb[i] - q.y0[i]) * ray_scale : q.yb[i]);
        if (threadIdx.x == 0) {
            double *r = a.res + (size_t)b * 12;
            r[0] = P; r[1] = D; r[2] = rp; r[3] = rd; r[4] = rg; r[5] = kkt; r[6] = omega;
            r[7] = normq; r[8] = (double)(t + 1); r[9] = (double)restarts; r[10] = status; r[11] = 0.0;
        }
        __syncthreads();
    }
}

// Unrolled rAPDHG: exactly T iterations from zero; schedule recorded or
// replayed; checkpoints of (x, y, xbar, ybar) before every kCkpt-th iteration.
template <int BT, bool ONCHIP>
__global__ __launch_bounds__(BT) void k_bqp_unrolled(QArgs a, QOpts o) {
    extern __shared__ double qlds[];
    const int32_t xw = (a.n + 63) >> 6, yw = (a.m + 63) >> 6;
    const int64_t nck = (a.T + kCkpt - 1) / kCkpt;
    const size_t cks = 2 * (size_t)a.n + 2 * (size_t)a.m;
    for (;;) {
        const int32_t b = qnext<BT>(a.queue);
        if (b >= a.B) return;
        QI q = qinst(a, b);
        if (ONCHIP) q_onchip(a, q, qlds);
        double cn, bn, cnorm, bnorm;
        qprepare<BT>(a, q, cn, bn, cnorm, bnorm);
        qinit<BT>(a, q, nullptr, nullptr);
        const double normq = a.normq[b];
        double omega = (cn > 1e-10 && bn > 1e-10) ? cn / bn : 1.0;
        uint8_t *rs_ = a.restart + (size_t)b * a.T;
        double *om_ = a.omega + (size_t)b * a.T;
        int32_t *kk_ = a.kk + (size_t)b * a.T;
        double r_start = 0.0, r_prev = 0.0;
        int64_t k = 0;
        for (int64_t t = 0; t < a.T; ++t) {
            if (a.replay) omega = om_[t];
            if (t % kCkpt == 0) {
                double *ck = a.ckpt + ((size_t)b * nck + t / kCkpt) * cks;
                for (int32_t j = threadIdx.x; j < a.n; j += BT) {
                    ck[j] = q.x[j];
                    ck[a.n + j] = q.xb[j];
                }
                for (int32_t i = threadIdx.x; i < a.m; i += BT) {
                    ck[2 * a.n + i] = q.y[i];
                    ck[2 * a.n + a.m + i] = q.yb[i];
                }
            }
            uint64_t *xmt = a.xmask + ((size_t)b * a.T + t) * xw;
            uint64_t *ymt = a.ymask + ((size_t)b * a.T + t) * 2 * yw;
            qstep<BT>(a, q, k, omega, normq, xmt, ymt);
            if (a.vall)
                for (int32_t j = threadIdx.x; j < a.n; j += BT) a.vall[((size_t)b * a.T + t) * a.n + j] = q.v[j];
            if (threadIdx.x == 0) {
                om_[t] = omega;
                kk_[t] = (int32_t)k;
            }
            if (t + 1 >= a.T) break;
            bool restart = a.replay ? rs_[t] != 0 : false;
            if (!a.replay && (t % o.check_every) == 0) {
                double v[8];
                qcheck<BT>(a, q, v);
                const double P = 0.5 * v[2] + v[3];
                const double D = -0.5 * v[2] + v[6] + v[4];
                const double ap = sqrt(v[5]), ad = sqrt(v[1]), ag = fabs(P - D);
                const double r = sqrt(omega * ap * ap + ad * ad / omega + ag * ag);
                if (t == 0) {
                    r_start = r;
                    r_prev = r;
                } else if (r <= o.beta_suff * r_start || (r <= o.beta_nec * r_start && r > r_prev) ||
                           (double)k >= o.beta_art * (double)t) {
                    restart = true;
                } else {
                    r_prev = r;
                }
                if (restart) {
                    const double dxr = sqrt(v[0]), dyr = sqrt(v[7]);
                    omega = batch_new_omega(omega, dxr, dyr);
                    r_start = r;
                    r_prev = r;
                }
            }
            if (threadIdx.x == 0 && !a.replay) rs_[t] = restart ? 1 : 0;
            if (restart) {
                qrestart<BT>(a, q);
                k = 0;
            } else {
                ++k;
            }
        }
        if (threadIdx.x == 0 && !a.replay) rs_[a.T - 1] = 0;
        for (int32_t j = threadIdx.x; j < a.n; j += BT) a.x_out[(size_t)b * a.n + j] = a.Dc[j] * q.xb[j];
        for (int32_t i = threadIdx.x; i < a.m; i += BT) a.y_out[(size_t)b * a.m + i] = a.Dr[i] * q.yb[i];
        __syncthreads();
    }
}

// Reverse pass of k_bqp_unrolled: per segment, recompute the momentum points
// from the checkpoint, then walk the segment backwards.
template <int BT, bool ONCHIP>
__global__ __launch_bounds__(BT) void k_bqp_backward(QArgs a, QOpts o) {
    extern __shared__ double qlds[];
    const int32_t xw = (a.n + 63) >> 6, yw = (a.m + 63) >> 6;
    const int64_t nck = (a.T + kCkpt - 1) / kCkpt;
    const size_t cks = 2 * (size_t)a.n + 2 * (size_t)a.m;
    for (;;) {
        const int32_t b = qnext<BT>(a.queue);
        if (b >= a.B) return;
        QI q = qinst(a, b);
        if (ONCHIP) q_onchip(a, q, qlds);
        double cn, bn, cnorm, bnorm;
        qprepare<BT>(a, q, cn, bn, cnorm, bnorm);
        const double normq = a.normq[b];
        const uint8_t *rs_ = a.restart + (size_t)b * a.T;
        const double *om_ = a.omega + (size_t)b * a.T;
        const int32_t *kk_ = a.kk + (size_t)b * a.T;
        double *vseg = a.vseg + (size_t)b * kCkpt * a.n;
        // cotangents: bx (x), by (y), bxb, byb; scratch bw (m), bqv (n), xe holds bxe
        double *bx = q.x0, *by = q.y0;
        double *bxb = a.bxb + (size_t)b * a.n, *byb = a.byb + (size_t)b * a.m;
        double *bw = a.bw + (size_t)b * a.m, *bqv = a.bqv + (size_t)b * a.n;
        if (ONCHIP) {
            // after the 9 n- and 5 m-vectors of q_onchip
            double *p = qlds + 9 * (size_t)a.n + 5 * (size_t)a.m;
            bxb = p; p += a.n;
            bqv = p; p += a.n;
            byb = p; p += a.m;
            bw = p;
        }
        double *gc = a.gc + (size_t)b * a.n, *gd = a.gd + (size_t)b * a.n;
        double *glc = a.glc + (size_t)b * a.m, *guc = a.guc + (size_t)b * a.m;
        for (int32_t j = threadIdx.x; j < a.n; j += BT) {
            bx[j] = 0.0;
            bxb[j] = a.Dc[j] * a.gx[(size_t)b * a.n + j];
            gc[j] = 0.0;
            gd[j] = 0.0;
        }
        for (int32_t i = threadIdx.x; i < a.m; i += BT) {
            by[i] = 0.0;
            byb[i] = a.Dr[i] * (a.gy ? a.gy[(size_t)b * a.m + i] : 0.0);
            glc[i] = 0.0;
            guc[i] = 0.0;
        }
        __syncthreads();
        for (int64_t seg = nck - 1; seg >= 0; --seg) {
            const int64_t t0 = seg * kCkpt, t1 = min(a.T, t0 + kCkpt);
            // recompute the segment's momentum points from the checkpoint,
            // unless the forward kept them all
            if (!a.vall) {
                const double *ck = a.ckpt + ((size_t)b * nck + seg) * cks;
                for (int32_t j = threadIdx.x; j < a.n; j += BT) {
                    q.x[j] = ck[j];
                    q.xb[j] = ck[a.n + j];
                }
                for (int32_t i = threadIdx.x; i < a.m; i += BT) {
                    q.y[i] = ck[2 * a.n + i];
                    q.yb[i] = ck[2 * a.n + a.m + i];
                }
                __syncthreads();
                for (int64_t t = t0; t < t1; ++t) {
                    qstep<BT>(a, q, kk_[t], om_[t], normq, nullptr, nullptr);
                    for (int32_t j = threadIdx.x; j < a.n; j += BT) vseg[(size_t)(t - t0) * a.n + j] = q.v[j];
                    if (t + 1 < a.T && rs_[t]) {
                        for (int32_t j = threadIdx.x; j < a.n; j += BT) q.x[j] = q.xb[j];
                        for (int32_t i = threadIdx.x; i < a.m; i += BT) q.y[i] = q.yb[i];
                    }
                    __syncthreads();
                }
            }
            for (int64_t t = t1 - 1; t >= t0; --t) {
                if (t < a.T - 1 && rs_[t]) {
                    for (int32_t j = threadIdx.x; j < a.n; j += BT) {
                        bxb[j] += bx[j];
                        bx[j] = 0.0;
                    }
                    for (int32_t i = threadIdx.x; i < a.m; i += BT) {
                        byb[i] += by[i];
                        by[i] = 0.0;
                    }
                    __syncthreads();
                }
                const int64_t k = kk_[t];
                const double omega = om_[t];
                const double beta = 2.0 / (double)(k + 2), theta = beta;
                const double tau = 1.0 / (omega / a.eta + 2.0 * normq / (double)(k + 1));
                const double sigma = a.eta * omega;
                const uint64_t *xmt = a.xmask + ((size_t)b * a.T + t) * xw;
                const uint64_t *ymt = a.ymask + ((size_t)b * a.T + t) * 2 * yw;
                // averages and the dual step (bx holds bx+ after this loop)
                for (int32_t j = threadIdx.x; j < a.n; j += BT) {
                    bx[j] = bx[j] + theta * bxb[j];
                    bxb[j] = (1.0 - theta) * bxb[j];
                }
                for (int32_t i = threadIdx.x; i < a.m; i += BT) {
                    const double byp = by[i] + theta * byb[i];
                    byb[i] = (1.0 - theta) * byb[i];
                    const uint64_t bit = 1ull << (i & 63);
                    const bool at_u = (ymt[2 * (i >> 6)] & bit) != 0;
                    const bool at_l = (ymt[2 * (i >> 6) + 1] & bit) != 0;
                    const double w = (at_u || at_l) ? sigma * byp : 0.0;
                    if (at_u) guc[i] += sigma * byp;
                    if (at_l) glc[i] += sigma * byp;
                    by[i] = w / sigma;
                    bw[i] = -w;
                }
                __syncthreads();
                // xe = 2x+ - x, primal step
                for (int32_t j = threadIdx.x; j < a.n; j += BT) {
                    const double bxe = qdot(a.trp, a.tci, a.tva, j, bw);
                    const double bxp = bx[j] + 2.0 * bxe;
                    const bool inside = (xmt[j >> 6] >> (j & 63)) & 1ull;
                    const double bu = inside ? bxp : 0.0;
                    bx[j] = -bxe + bu;
                    bqv[j] = -tau * bu;
                    gc[j] += -tau * bu;
                    q.xe[j] = tau * bu;
                }
                __syncthreads();
                if (a.wave_rows) {
                    for (int32_t i = (int32_t)(threadIdx.x >> 6); i < a.m; i += BT / 64) {
                        const double s = qdot_wave(a.arp, a.aci, a.ava, i, q.xe);
                        if ((threadIdx.x & 63) == 0) by[i] += s;
                    }
                } else {
                    for (int32_t i = threadIdx.x; i < a.m; i += BT) by[i] += qdot(a.arp, a.aci, a.ava, i, q.xe);
                }
                // Q~ v: bv = F~ (F~' bqv) + d~ bqv, gradient in d~
                const double *t2 = qt_of<BT>(a, bqv);
                const double *vt = a.vall ? a.vall + ((size_t)b * a.T + t) * a.n : vseg + (size_t)(t - t0) * a.n;
                for (int32_t j = threadIdx.x; j < a.n; j += BT) {
                    const double bv = qv_row(a, q, j, t2, bqv);
                    gd[j] += bqv[j] * vt[j];
                    bxb[j] += (1.0 - beta) * bv;
                    bx[j] += beta * bv;
                }
                __syncthreads();
            }
        }
        for (int32_t j = threadIdx.x; j < a.n; j += BT) {
            const double d = a.Dc[j];
            gc[j] = d * gc[j];
            gd[j] = (d * d) * gd[j];
        }
        for (int32_t i = threadIdx.x; i < a.m; i += BT) {
            glc[i] = isfinite(q.lc_o[i]) ? a.Dr[i] * glc[i] : 0.0;
            guc[i] = isfinite(q.uc_o[i]) ? a.Dr[i] * guc[i] : 0.0;
        }
        __syncthreads();
    }
}

// F~' = (D_c F)' stored [r_pad][n] (rows from r on stay zero) from F [n][r];
// flags non-finite entries.
__global__ __launch_bounds__(kBlock) void k_bqp_scale_factor(int32_t n, int32_t r,
                                                             const double *__restrict__ Dc,
                                                             const double *__restrict__ F,
                                                             double *__restrict__ Fo,
                                                             int32_t *__restrict__ flag) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * r) return;
    const int64_t j = t / r, p = t % r;
    if (!isfinite(F[t])) atomicOr(flag, 1);
    Fo[p * n + j] = Dc[j] * F[t];
}

}  // namespace pdhg

// ---------------------------------------------------------------------------
// host side

#include "batch_internal.hpp"

namespace pdhg {

static QOpts qopts(const pdhg_options &o) {
    QOpts q;
    q.eps = o.eps;
    q.gamma = o.gamma;
    q.beta_suff = o.restart_sufficient;
    q.beta_nec = o.restart_necessary;
    q.beta_art = o.restart_artificial;
    q.power_tol = o.power_tol;
    q.limit = std::min<int64_t>(o.iteration_limit, 10000000);
    q.check_every = o.check_every;
    q.power_max_iters = o.power_max_iters;
    q.eps_pinf = o.eps_primal_infeasible;
    q.eps_dinf = o.eps_dual_infeasible;
    q.detect = o.eps_primal_infeasible > 0.0 || o.eps_dual_infeasible > 0.0;
    q.pad = 0;
    return q;
}

static QArgs qargs(BatchHandle &h) {
    QArgs a;
    memset(&a, 0, sizeof(a));
    a.B = h.B;
    a.m = h.m;
    a.n = h.n;
    a.r = h.q_rank;
    // one wave per row when the rows are few and long (e.g. a budget row)
    a.wave_rows = (h.m <= kWaveRowsMax && h.m > 0 && h.nnz >= (int64_t)32 * h.m) ? 1 : 0;
    a.arp = h.arp.p;
    a.aci = h.aci.p;
    a.trp = h.trp.p;
    a.tci = h.tci.p;
    a.ava = h.ava.p;
    a.tva = h.tva.p;
    a.Dr = h.Dr.p;
    a.Dc = h.Dc.p;
    a.eta = h.q_eta;
    a.FT = h.qF.p;
    a.d_o = h.qd_o.p;
    a.normq = h.normq.p;
    a.c_o = h.c_o.p;
    a.lc_o = h.lc_o.p;
    a.uc_o = h.uc_o.p;
    a.lv_o = h.lv_o.p;
    a.uv_o = h.uv_o.p;
    a.c = h.c.p;
    a.lc = h.lc.p;
    a.uc = h.uc.p;
    a.lv = h.lv.p;
    a.uv = h.uv.p;
    a.dd = h.qdd.p;
    a.x = h.x.p;
    a.y = h.y.p;
    a.xb = h.xbar.p;
    a.yb = h.ybar.p;
    a.x0 = h.x0.p;
    a.y0 = h.y0.p;
    a.xe = h.xe.p;
    a.v = h.qv_.p;
    a.res = h.qres.p;
    a.queue = h.queue.p;
    a.T = h.unrolled_T;
    a.restart = h.u_restart.p;
    a.omega = h.u_omega.p;
    a.kk = h.u_kk.p;
    a.xmask = h.u_xmask.p;
    a.ymask = h.u_ymask.p;
    a.ckpt = h.ckpt.p;
    a.vseg = h.vseg.p;
    a.vall = h.u_vall ? h.vall.p : nullptr;
    a.bxb = h.bxb.p;
    a.byb = h.byb.p;
    a.bw = h.bw.p;
    a.bqv = h.bqv.p;
    return a;
}

template <class K>
static int32_t q_wgs(BatchHandle &h, K kernel, int BT, size_t lds = 0) {
    int per_cu = 0;
    PDHG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kernel), BT, lds));
    int32_t wg = std::min(h.B, std::max(1, per_cu) * h.q_cus);
    if (h.workgroups > 0) wg = std::min(wg, h.workgroups);
    return wg;
}

enum class QK { norm, solve, unrolled, backward };

template <int BT>
static void qlaunch_t(BatchHandle &h, QK which, const QArgs &a, const QOpts &o) {
    PDHG_HIP(hipMemsetAsync(h.queue.p, 0, sizeof(int32_t), h.stream));
    switch (which) {
        case QK::norm:
            k_bqp_norm<BT><<<q_wgs(h, k_bqp_norm<BT>, BT), BT, 0, h.stream>>>(a, o);
            break;
        case QK::solve:
            // the ray pass costs registers: kernels without it when the tests are off
            if (q_onchip_bytes(a.n, a.m) <= kQOnchipBytes) {
                const size_t l = q_onchip_bytes(a.n, a.m);
                if (o.detect)
                    k_bqp_solve<BT, true, true><<<q_wgs(h, k_bqp_solve<BT, true, true>, BT, l), BT, l, h.stream>>>(a, o);
                else
                    k_bqp_solve<BT, false, true><<<q_wgs(h, k_bqp_solve<BT, false, true>, BT, l), BT, l, h.stream>>>(a, o);
            } else if (o.detect) {
                k_bqp_solve<BT, true, false><<<q_wgs(h, k_bqp_solve<BT, true, false>, BT), BT, 0, h.stream>>>(a, o);
            } else {
                k_bqp_solve<BT, false, false><<<q_wgs(h, k_bqp_solve<BT, false, false>, BT), BT, 0, h.stream>>>(a, o);
            }
            break;
        case QK::unrolled: {
            const size_t l = q_onchip_bytes(a.n, a.m);
            if (l <= kQOnchipBytes)
                k_bqp_unrolled<BT, true><<<q_wgs(h, k_bqp_unrolled<BT, true>, BT, l), BT, l, h.stream>>>(a, o);
            else
                k_bqp_unrolled<BT, false><<<q_wgs(h, k_bqp_unrolled<BT, false>, BT), BT, 0, h.stream>>>(a, o);
            break;
        }
        case QK::backward: {
            const size_t l = q_onchip_bytes_bwd(a.n, a.m);
            if (l <= kQOnchipBytes)
                k_bqp_backward<BT, true><<<q_wgs(h, k_bqp_backward<BT, true>, BT, l), BT, l, h.stream>>>(a, o);
            else
                k_bqp_backward<BT, false><<<q_wgs(h, k_bqp_backward<BT, false>, BT), BT, 0, h.stream>>>(a, o);
            break;
        }
    }
    PDHG_HIP(hipGetLastError());
    PDHG_HIP(hipStreamSynchronize(h.stream));
}

static void qlaunch(BatchHandle &h, QK which, const QArgs &a) {
    const QOpts o = qopts(h.opt);
    // the QP kernels spill registers at 1024 threads: at most 512 unless the
    // caller chose the shape
    const int32_t threads = h.threads_set ? h.threads : std::min(h.threads, 512);
    switch (threads) {
        case 64: qlaunch_t<64>(h, which, a, o); break;
        case 128: qlaunch_t<128>(h, which, a, o); break;
        case 512: qlaunch_t<512>(h, which, a, o); break;
        case 1024: qlaunch_t<1024>(h, which, a, o); break;
        default: qlaunch_t<256>(h, which, a, o); break;
    }
}

void bqp_create(BatchHandle &h, const pdhg_batch_problem &p) {
    hipStream_t s = h.stream;
    if (!h.shared) fail(PDHG_ERR_UNSUPPORTED, "QP batches need a shared constraint matrix");
    if (p.q_rank < 1 || p.q_rank > kRmax || !p.q_factor || !p.q_diag)
        fail(PDHG_ERR_INVALID_ARG, "QP batches need 1 <= q_rank <= 32, q_factor and q_diag");
    h.q_rank = p.q_rank;
    {
        int dev = 0, cus = 0;
        PDHG_HIP(hipGetDevice(&dev));
        PDHG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        h.q_cus = std::max(1, cus);
        // eta depends on A only: read once (the setup launch has completed)
        PDHG_HIP(hipMemcpy(&h.q_eta, h.eta.p, sizeof(double), hipMemcpyDeviceToHost));
    }
    const size_t nf = (size_t)h.n * h.q_rank;
    DBuf<double> F;
    F.alloc(nf);
    h.qd_o.alloc((size_t)h.vec_n);
    const hipMemcpyKind kind = p.mem == PDHG_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    PDHG_HIP(hipMemcpyAsync(F.p, p.q_factor, nf * sizeof(double), kind, s));
    PDHG_HIP(hipMemcpyAsync(h.qd_o.p, p.q_diag, (size_t)h.vec_n * sizeof(double), kind, s));
    DBuf<int32_t> flag;
    flag.alloc(1);
    PDHG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    // F~' [r_pad][n] with zero rows r..r_pad-1 (r_pad = r rounded up to 8)
    const size_t nfp = (size_t)h.n * (size_t)((h.q_rank + 7) & ~7);
    h.qF.alloc(nfp);
    PDHG_HIP(hipMemsetAsync(h.qF.p, 0, nfp * sizeof(double), s));
    k_bqp_scale_factor<<<(unsigned)std::max<int64_t>(1, ceil_div((int64_t)nf, kBlock)), kBlock, 0, s>>>(
        h.n, h.q_rank, h.Dc.p, F.p, h.qF.p, flag.p);
    check_flag(s, flag.p, "non-finite entry in the factor of Q");
    // d is validated as a vector of bounds would be: finite
    validate_vectors(s, h.vec_n, 0, h.qd_o.p, h.lv_o.p, h.uv_o.p, nullptr, nullptr);
    for (auto *b : {&h.qdd, &h.xbar, &h.qv_}) b->alloc((size_t)h.vec_n);
    h.ybar.alloc((size_t)std::max(1, h.vec_m));
    h.normq.alloc((size_t)h.B);
    h.qres.alloc((size_t)h.B * 12);
    QArgs a = qargs(h);
    qlaunch(h, QK::norm, a);
}

void bqp_solve(BatchHandle &h, const double *x_init, const double *y_init, double *x_out,
               double *y_out, pdhg_result *res) {
    const double t0 = now_seconds();
    QArgs a = qargs(h);
    a.x_init = x_init;
    a.y_init = y_init;
    a.x_out = x_out;
    a.y_out = y_out;
    qlaunch(h, QK::solve, a);
    const double el = now_seconds() - t0;
    if (res) {
        std::vector<double> r((size_t)h.B * 12);
        PDHG_HIP(hipMemcpy(r.data(), h.qres.p, r.size() * 8, hipMemcpyDeviceToHost));
        for (int32_t b = 0; b < h.B; ++b) {
            const double *q = &r[(size_t)b * 12];
            pdhg_result &o = res[b];
            memset(&o, 0, sizeof(o));
            o.primal_obj = q[0];
            o.dual_obj = q[1];
            o.rel_primal_res = q[2];
            o.rel_dual_res = q[3];
            o.rel_gap = q[4];
            o.kkt_rel = q[5];
            o.omega = q[6];
            o.norm_q = q[7];
            o.iterations = (int64_t)q[8];
            o.restarts = (int64_t)q[9];
            o.status = (int32_t)q[10];
            o.solve_seconds = el;
            o.setup_seconds = h.setup_seconds;
            o.eta = a.eta;
        }
    }
}

void bqp_unrolled(BatchHandle &h, int64_t T, int32_t replay, double *x_out, double *y_out) {
    if (T < 1 || T > 1000000) fail(PDHG_ERR_INVALID_ARG, "T must be in [1, 10^6]");
    if (replay && h.unrolled_T != T)
        fail(PDHG_ERR_INVALID_ARG, "replay needs a recorded schedule of the same length T");
    if (h.unrolled_T != T) {
        const int64_t xw = (h.n + 63) / 64, yw = (h.m + 63) / 64;
        const int64_t nck = (T + kCkpt - 1) / kCkpt;
        h.u_xmask.alloc((size_t)std::max<int64_t>(1, (int64_t)h.B * T * xw));
        h.u_ymask.alloc((size_t)std::max<int64_t>(1, (int64_t)h.B * T * 2 * yw));
        h.u_restart.alloc((size_t)h.B * T);
        h.u_omega.alloc((size_t)h.B * T);
        h.u_kk.alloc((size_t)h.B * T);
        h.ckpt.alloc((size_t)h.B * nck * (2 * (size_t)h.n + 2 * (size_t)h.m));
        h.vseg.alloc((size_t)h.B * kCkpt * h.n);
        // on-chip instances keep every momentum point (at most 16 GiB), so the
        // reverse pass needs no recomputation; larger ones recompute segments
        const size_t vbytes = (size_t)h.B * (size_t)T * (size_t)h.n * sizeof(double);
        h.u_vall = q_onchip_bytes_bwd(h.n, h.m) <= kQOnchipBytes && vbytes <= ((size_t)16 << 30);
        if (h.u_vall)
            h.vall.alloc((size_t)h.B * (size_t)T * (size_t)h.n);
        else
            h.vall.release();
        h.bxb.alloc((size_t)h.vec_n);
        h.bqv.alloc((size_t)h.vec_n);
        h.byb.alloc((size_t)std::max(1, h.vec_m));
        h.bw.alloc((size_t)std::max(1, h.vec_m));
        h.unrolled_T = T;
    }
    QArgs a = qargs(h);
    a.replay = replay;
    a.x_out = x_out;
    a.y_out = y_out;
    qlaunch(h, QK::unrolled, a);
}

void bqp_backward(BatchHandle &h, const double *gx, const double *gy, double *gc, double *glc,
                  double *guc, double *gd) {
    if (h.unrolled_T < 1) fail(PDHG_ERR_INVALID_ARG, "run pdhg_batch_unrolled_forward first");
    DBuf<double> lcs, ucs, ds;
    lcs.alloc((size_t)std::max(1, h.vec_m));
    ucs.alloc((size_t)std::max(1, h.vec_m));
    ds.alloc((size_t)h.vec_n);
    QArgs a = qargs(h);
    a.gx = gx;
    a.gy = gy;
    a.gc = gc;
    a.glc = glc ? glc : lcs.p;
    a.guc = guc ? guc : ucs.p;
    a.gd = gd ? gd : ds.p;
    qlaunch(h, QK::backward, a);
}

}  // namespace pdhg
