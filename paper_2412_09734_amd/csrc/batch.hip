// Batched r2HPDHG (MPAX paper, Section 3 "Batched solving"; Algorithm 1).
//
// One workgroup owns one LP instance at a time and runs its whole solve:
// scaling and power iteration (setup kernel), then the iteration loop with
// checks, restarts and early exit (solve kernel). Workgroups take instances
// from a queue (an integer counter) until the batch is exhausted, so a launch
// of as many workgroups as the GPU holds covers any batch size. Every
// reduction is a fixed-order workgroup tree, so an instance's result does not
// depend on which workgroup ran it.
//
// Matrices are plain CSR (rows in original order) with instance-local column
// indices; row pointers hold global entry offsets. Per-instance vectors live
// in HBM and stay in L2 while the instance runs.
#include <algorithm>
#include <climits>
#include <memory>
#include <vector>

#include "device.hpp"
#include "batch_internal.hpp"

namespace pdhg {

struct BOpts {
    double eps, gamma, step_safety, beta_suff, beta_nec, beta_art, power_tol;
    int64_t limit;
    int32_t check_every, ruiz_iters, pock_chambolle, power_max_iters;
    double eps_pinf, eps_dinf;   // infeasibility certificate tolerances
    int32_t detect, pad;         // 1: test the rays at checks
};

struct BArgs {
    int32_t B, shared, m, n;
    const int32_t *row_off, *col_off;
    const int32_t *arp, *aci;
    double *ava;
    const int32_t *trp, *tci;
    double *tva;
    double *Dr, *Dc, *eta;
    int32_t *power_iters;
    const double *c_o, *lc_o, *uc_o, *lv_o, *uv_o;
    double *c, *lc, *uc, *lv, *uv;
    double *x, *x0, *xh, *xe, *aty, *y, *y0, *yh;
    const double *x_init, *y_init;
    double *x_out, *y_out;
    BatchRes *res;
    int32_t *queue;
    // SELL-64 copies (entry k of local row i at sp[sfirst + i/64] + 64 k + i%64)
    const int32_t *asp, *asci, *asfirst, *tsp, *tsci, *tsfirst;
    const double *asva, *tsva;
    double *lhist;    // Lanczos alpha / beta per instance, stride 2 (power_max_iters + 1)
    // infeasibility rays: the anchor's products A~x0 (like y), A~'y0 (like x)
    // and this check's A~xhat, A~'yhat
    double *p0, *q0, *ph, *qh;
};

// Geometry of instance b: matrix rows start at r0 (A) / c0 (A'); vectors at
// vr / vc; scaling vectors at dr / dc.
struct Geo {
    int32_t m, n, r0, c0, vr, vc, dr, dc, sidx;
};

__device__ __forceinline__ Geo geometry(const BArgs &a, int32_t b) {
    Geo g;
    if (a.shared) {
        g.m = a.m;
        g.n = a.n;
        g.r0 = 0;
        g.c0 = 0;
        g.vr = b * a.m;
        g.vc = b * a.n;
        g.dr = 0;
        g.dc = 0;
        g.sidx = 0;
    } else {
        g.r0 = a.row_off[b];
        g.c0 = a.col_off[b];
        g.m = a.row_off[b + 1] - g.r0;
        g.n = a.col_off[b + 1] - g.c0;
        g.vr = g.r0;
        g.vc = g.c0;
        g.dr = g.r0;
        g.dc = g.c0;
        g.sidx = b;
    }
    return g;
}

// Deterministic workgroup sum of K values per thread, result in every thread:
// wave butterflies, then thread q adds the wave totals of value q in wave
// order (one value per thread keeps the register footprint independent of
// the workgroup size).
template <int BT, int K>
__device__ __forceinline__ void wg_sum(double (&v)[K]) {
    constexpr int NW = BT / 64;
    __shared__ double sh[K][NW];
    __shared__ double tot[K];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) sh[q][wave] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < K) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += sh[threadIdx.x][w];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = tot[q];
    __syncthreads();
}

// Workgroup maxima of K values (order-free), result in every thread.
template <int BT, int K>
__device__ __forceinline__ void wg_max(double (&v)[K]) {
    constexpr int NW = BT / 64;
    __shared__ double sh[K][NW];
    __shared__ double tot[K];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double s = wave_max(v[q]);
        if (lane == 0) sh[q][wave] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < K) {
        double s = sh[threadIdx.x][0];
        for (int w = 1; w < NW; ++w) s = fmax(s, sh[threadIdx.x][w]);
        tot[threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = tot[q];
    __syncthreads();
}

template <int BT>
__device__ __forceinline__ int32_t next_instance(int32_t *queue) {
    __shared__ int32_t id;
    if (threadIdx.x == 0) id = atomicAdd(queue, 1);
    __syncthreads();
    // the same value in every lane: a scalar, so the instance's pointers and
    // sizes live in scalar registers
    const int32_t r = __builtin_amdgcn_readfirstlane(id);
    __syncthreads();
    return r;
}

// CSR row dot product, entries added in row order; four entries' loads (and
// then their gathers) are issued before their products, so a thread's walk
// over the row waits on a quarter as many round trips.
__device__ __forceinline__ double csr_dot(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                          const double *__restrict__ va, int32_t row,
                                          const double *__restrict__ v) {
    double acc = 0.0;
    int32_t e = rp[row];
    const int32_t e1 = rp[row + 1];
    for (; e + 4 <= e1; e += 4) {
        int32_t c[4];
        double a[4], x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c[q] = ci[e + q];
            a[q] = va[e + q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = v[c[q]];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc = fma(a[q], x[q], acc);
    }
    for (; e < e1; ++e) acc = fma(va[e], v[ci[e]], acc);
    return acc;
}

// Ruiz / Pock-Chambolle factor of one CSR row: max |a| (pc = false) or the sum
// of |a| (pc = true) over the row in entry order, loads four at a time.
__device__ __forceinline__ double csr_absnorm(const int32_t *__restrict__ rp, const double *__restrict__ va,
                                              int32_t row, bool pc) {
    double acc = 0.0;
    int32_t e = rp[row];
    const int32_t e1 = rp[row + 1];
    for (; e + 4 <= e1; e += 4) {
        double a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = fabs(va[e + q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc = pc ? acc + a[q] : fmax(acc, a[q]);
    }
    for (; e < e1; ++e) acc = pc ? acc + fabs(va[e]) : fmax(acc, fabs(va[e]));
    return acc;
}

// va[e] /= (r * f[ci[e]]) over CSR row `row`, four entries at a time.
__device__ __forceinline__ void csr_rescale(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                            double *__restrict__ va, int32_t row, double r,
                                            const double *__restrict__ f) {
    int32_t e = rp[row];
    const int32_t e1 = rp[row + 1];
    for (; e + 4 <= e1; e += 4) {
        int32_t c[4];
        double a[4], x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c[q] = ci[e + q];
            a[q] = va[e + q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = f[c[q]];
#pragma unroll
        for (int q = 0; q < 4; ++q) va[e + q] = a[q] / (r * x[q]);
    }
    for (; e < e1; ++e) va[e] = va[e] / (r * f[ci[e]]);
}

// Row sum of a SELL-64 slice row: lane `lane` of slice `sl`; entries walked in
// row order (padding entries are (column 0, value 0.0)).
__device__ __forceinline__ double sell_dot_bw(const int32_t *__restrict__ ci, const double *__restrict__ va,
                                              int32_t base, int32_t w, int32_t lane,
                                              const double *__restrict__ v);

__device__ __forceinline__ double sell_dot(const int32_t *__restrict__ sp, const int32_t *__restrict__ ci,
                                           const double *__restrict__ va, int32_t sl, int32_t lane,
                                           const double *__restrict__ v) {
    const int32_t b = sp[sl], w = (sp[sl + 1] - b) >> 6;
    return sell_dot_bw(ci, va, b, w, lane, v);
}

// Same with the slice's first entry and width already known. Entries are
// fetched four at a time before they are used (independent loads in flight),
// and added in row order.
__device__ __forceinline__ double sell_dot_bw(const int32_t *__restrict__ ci, const double *__restrict__ va,
                                              int32_t base, int32_t w, int32_t lane,
                                              const double *__restrict__ v) {
    double acc = 0.0;
    int32_t k = 0;
    for (; k + 4 <= w; k += 4) {
        int32_t c[4];
        double a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t e = base + 64 * (k + q) + lane;
            c[q] = ci[e];
            a[q] = va[e];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc = fma(a[q], v[c[q]], acc);
    }
    if (k + 2 <= w) {
        const int32_t e0 = base + 64 * k + lane, e1 = e0 + 64;
        const int32_t c0 = ci[e0], c1 = ci[e1];
        const double a0 = va[e0], a1 = va[e1];
        acc = fma(a0, v[c0], acc);
        acc = fma(a1, v[c1], acc);
        k += 2;
    }
    if (k < w) {
        const int32_t e = base + 64 * k + lane;
        acc = fma(va[e], v[ci[e]], acc);
    }
    return acc;
}

__device__ __forceinline__ uint64_t splitmix64_b(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// setup: Ruiz + Pock-Chambolle scaling and the power iteration, per instance
// (once for a shared matrix).

// Sturm count of T - x I for T = B'B, B the Golub-Kahan bidiagonal (alpha on
// the diagonal, beta above it): the number of negative pivots of the LDL'
// recurrence, i.e. the number of eigenvalues of T below x.
__device__ int32_t bidiag_sturm(const double *alpha, const double *beta, int32_t k, double x) {
    int32_t cnt = 0;
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

// Largest eigenvalue of T = B'B: bisection over [0, Gershgorin bound], at most
// 200 halvings, until the interval cannot be halved. The whole workgroup takes
// D = log2(BT) halvings per round: thread t (1 <= t < BT) replays the midpoint
// arithmetic along the path to node t of the binary tree of the next D
// midpoints (bit 0: upper half dropped, bit 1: lower half dropped) and counts
// at its own midpoint; thread 0 then walks the tree from the root. The result
// equals the one-point-at-a-time bisection bit for bit.
template <int BT>
__device__ double bidiag_lambda_max_wg(const double *alpha, const double *beta, int32_t k) {
    constexpr int NW = BT / 64;
    constexpr int D = BT == 64 ? 6 : BT == 128 ? 7 : BT == 256 ? 8 : BT == 512 ? 9 : 10;
    static_assert((1 << D) == BT, "BT must be a power of two from 64 to 1024");
    __shared__ double wmax[NW];
    __shared__ double lohi[2];
    __shared__ int32_t done;
    __shared__ uint8_t halvable[BT], lower[BT];
    const int32_t t = threadIdx.x;
    // Gershgorin bound: a maximum, the same in any order
    double g = 0.0;
    for (int32_t i = t; i < k; i += BT) {
        const double di = alpha[i] * alpha[i] + (i > 0 ? beta[i - 1] * beta[i - 1] : 0.0);
        const double el = i > 0 ? fabs(alpha[i - 1] * beta[i - 1]) : 0.0;
        const double er = i + 1 < k ? fabs(alpha[i] * beta[i]) : 0.0;
        g = fmax(g, di + el + er);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) g = fmax(g, __shfl_xor(g, off));
    if ((t & 63) == 0) wmax[t >> 6] = g;
    __syncthreads();
    double hi = 0.0;
    for (int w = 0; w < NW; ++w) hi = fmax(hi, wmax[w]);
    double lo = 0.0;
    int32_t halvings = 0;
    for (;;) {
        if (t > 0) {
            const int depth = 31 - __clz(t);
            double l = lo, h = hi;
            bool reach = true;
            for (int lev = depth - 1; lev >= 0; --lev) {
                const double mid = 0.5 * (l + h);
                if (!(mid > l && mid < h)) {
                    reach = false;
                    break;
                }
                if ((t >> lev) & 1) l = mid;
                else h = mid;
            }
            bool hv = false, lw = false;
            if (reach) {
                const double mid = 0.5 * (l + h);
                hv = mid > l && mid < h;
                if (hv) lw = bidiag_sturm(alpha, beta, k, mid) == k;
            }
            halvable[t] = hv;
            lower[t] = lw;
        }
        __syncthreads();
        if (t == 0) {
            int32_t node = 1, stop = 0;
            for (int lev = 0; lev < D; ++lev) {
                if (halvings >= 200 || !halvable[node]) {
                    stop = 1;
                    break;
                }
                const double mid = 0.5 * (lo + hi);
                if (lower[node]) {   // every eigenvalue lies below mid
                    hi = mid;
                    node = 2 * node;
                } else {
                    lo = mid;
                    node = 2 * node + 1;
                }
                ++halvings;
            }
            lohi[0] = lo;
            lohi[1] = hi;
            done = stop || halvings >= 200;
        }
        __syncthreads();
        lo = lohi[0];
        hi = lohi[1];
        const bool fin = done != 0;
        __syncthreads();
        if (fin) break;
    }
    return hi;
}

// ONCHIP: the power iteration's gathered vectors v (n) and w (m) live in LDS.
template <int BT, bool ONCHIP>
__global__ __launch_bounds__(BT) void k_batch_setup(BArgs a, BOpts o, int32_t count, int32_t nmax) {
    extern __shared__ double lds[];
    for (;;) {
        const int32_t b = next_instance<BT>(a.queue);
        if (b >= count) return;
        const Geo g = geometry(a, b);
        const int32_t *arp = a.arp + g.r0, *trp = a.trp + g.c0;
        double *Dr = a.Dr + g.dr, *Dc = a.Dc + g.dc;
        double *rs = a.yh + g.vr, *cs = a.xh + g.vc;   // factor scratch
        for (int32_t i = threadIdx.x; i < g.m; i += BT) Dr[i] = 1.0;
        for (int32_t j = threadIdx.x; j < g.n; j += BT) Dc[j] = 1.0;
        const int passes = o.ruiz_iters + (o.pock_chambolle ? 1 : 0);
        for (int pass = 0; pass < passes; ++pass) {
            const bool pc = pass >= o.ruiz_iters;
            __syncthreads();
            for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                const double acc = csr_absnorm(arp, a.ava, i, pc);
                rs[i] = acc > 0.0 ? sqrt(acc) : 1.0;
            }
            for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                const double acc = csr_absnorm(trp, a.tva, j, pc);
                cs[j] = acc > 0.0 ? sqrt(acc) : 1.0;
            }
            __syncthreads();
            for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                Dr[i] = Dr[i] / rs[i];
                csr_rescale(arp, a.aci, a.ava, i, rs[i], cs);
            }
            for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                Dc[j] = Dc[j] / cs[j];
                csr_rescale(trp, a.tci, a.tva, j, cs[j], rs);
            }
        }
        __syncthreads();
        // ||A~||_2 by Golub-Kahan-Lanczos bidiagonalisation from the SplitMix64
        // start vector (see estimate_steps for the recurrences)
        int64_t nnz = (int64_t)arp[g.m] - arp[0];
        double lam = 0.0;
        int32_t it = 0;
        if (g.m > 0 && nnz > 0) {
            double *v = ONCHIP ? lds : a.xh + g.vc;          // gathered by rows
            double *u = ONCHIP ? lds + nmax : a.yh + g.vr;   // gathered by columns
            double *pr = a.y + g.vr, *qc = a.xe + g.vc;      // owner-only scratch
            double *al = a.lhist + (size_t)g.sidx * 2 * (o.power_max_iters + 1);
            double *be = al + (o.power_max_iters + 1);
            __shared__ double lam_sh;
            __shared__ int32_t stop_sh;
            double q0[1] = {0.0};
            for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                const double val = 0.5 + (double)(splitmix64_b((uint64_t)j) >> 11) * 0x1.0p-53;
                v[j] = val;
                q0[0] += val * val;
            }
            for (int32_t i = threadIdx.x; i < g.m; i += BT) u[i] = 0.0;
            wg_sum<BT, 1>(q0);
            const double nv = sqrt(q0[0]);
            for (int32_t j = threadIdx.x; j < g.n; j += BT) v[j] = v[j] / nv;
            __syncthreads();
            double lam_prev = 0.0, bprev = 0.0;
            for (it = 1; it <= o.power_max_iters; ++it) {
                double sp[1] = {0.0};
                for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                    const double pv = csr_dot(arp, a.aci, a.ava, i, v) - bprev * u[i];
                    pr[i] = pv;
                    sp[0] += pv * pv;
                }
                wg_sum<BT, 1>(sp);
                const double al_k = sqrt(sp[0]);
                if (!(al_k > 0.0)) {
                    if (it == 1) lam = 0.0;
                    break;
                }
                for (int32_t i = threadIdx.x; i < g.m; i += BT) u[i] = pr[i] / al_k;
                __syncthreads();
                double sq[1] = {0.0};
                for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                    const double qv = csr_dot(trp, a.tci, a.tva, j, u) - al_k * v[j];
                    qc[j] = qv;
                    sq[0] += qv * qv;
                }
                wg_sum<BT, 1>(sq);
                const double be_k = sqrt(sq[0]);
                if (threadIdx.x == 0) {
                    al[it - 1] = al_k;
                    be[it - 1] = be_k;
                }
                __syncthreads();
                const double l = bidiag_lambda_max_wg<BT>(al, be, it);
                if (threadIdx.x == 0) {
                    int32_t st = 0;
                    if (!(be_k > 0.0)) st = 1;
                    else if (it > 1 && fabs(l - lam_prev) <= o.power_tol * l) st = 1;
                    lam_sh = l;
                    stop_sh = st;
                }
                __syncthreads();
                lam = lam_sh;
                const bool stop = stop_sh != 0;
                __syncthreads();
                if (stop) break;
                lam_prev = lam;
                for (int32_t j = threadIdx.x; j < g.n; j += BT) v[j] = qc[j] / be_k;
                bprev = be_k;
                __syncthreads();
            }
            if (it > o.power_max_iters) it = o.power_max_iters;
        }
        if (threadIdx.x == 0) {
            const double na = sqrt(lam);
            a.eta[g.sidx] = na > 0.0 ? o.step_safety / na : 1.0;
            a.power_iters[g.sidx] = it;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// solve

// Infeasibility rays of instance g at a check (after its products were kept
// in qh / ph): sums rs = (dual-ray bound terms over the columns, c'dx,
// dual-ray bound terms over the rows) and maxima rm = (dual-ray violation,
// primal-ray violation), every thread receiving the totals, for the
// memory-resident k_batch_solve (a pass of its own there; x0 is read from
// memory). k_batch_solve_lds sums the same terms in the same order inside its
// check loops.
template <int BT>
__device__ __forceinline__ void batch_ray_pass(const BArgs &a, const Geo &g,
                                            const double *__restrict__ xh, const double *__restrict__ yh,
                                            const double *__restrict__ y0, double (&rs)[3], double (&rm)[2]) {
    const double *Dr = a.Dr + g.dr, *Dc = a.Dc + g.dc;
    const double *x0 = a.x0 + g.vc;
    double s[3] = {0.0, 0.0, 0.0}, mx[2] = {0.0, 0.0};
    // opaque thread index: the addresses below are formed here, not kept
    // live across the iteration loop the pass sits in
    int32_t t0 = (int32_t)threadIdx.x;
    asm volatile("" : "+v"(t0));
#pragma unroll 1
    for (int32_t j = t0; j < g.n; j += BT) {
        double s2[2], m2[2];
        ray_col_terms(a.qh[g.vc + j], a.q0[g.vc + j], Dc[j], xh[j] - x0[j], a.c_o[g.vc + j],
                      a.lv_o[g.vc + j], a.uv_o[g.vc + j], s2, m2);
        s[0] += s2[0];
        s[1] += s2[1];
        mx[0] = fmax(mx[0], m2[0]);
        mx[1] = fmax(mx[1], m2[1]);
    }
#pragma unroll 1
    for (int32_t i = t0; i < g.m; i += BT) {
        double s1[1], m2[2];
        ray_row_terms(a.ph[g.vr + i], a.p0[g.vr + i], Dr[i], yh[i] - y0[i], a.lc_o[g.vr + i],
                      a.uc_o[g.vr + i], s1, m2);
        s[2] += s1[0];
        mx[0] = fmax(mx[0], m2[0]);
        mx[1] = fmax(mx[1], m2[1]);
    }
    wg_sum<BT, 3>(s);
    wg_max<BT, 2>(mx);
    for (int q = 0; q < 3; ++q) rs[q] = s[q];
    rm[0] = mx[0];
    rm[1] = mx[1];
}

// RAYS: the checks also test infeasibility rays (a separate instantiation,
// so that solves without the test keep the leaner register budget).
template <int BT, bool RAYS>
__global__ __launch_bounds__(BT) void k_batch_solve(BArgs a, BOpts o) {
    for (;;) {
        const int32_t b = next_instance<BT>(a.queue);
        if (b >= a.B) return;
        const Geo g = geometry(a, b);
        const int32_t *arp = a.arp + g.r0, *trp = a.trp + g.c0;
        const int32_t *aci = a.aci, *tci = a.tci;
        const double *ava = a.ava, *tva = a.tva;
        const double *Dr = a.Dr + g.dr, *Dc = a.Dc + g.dc;
        const double *c_o = a.c_o + g.vc, *lv_o = a.lv_o + g.vc, *uv_o = a.uv_o + g.vc;
        const double *lc_o = a.lc_o + g.vr, *uc_o = a.uc_o + g.vr;
        double *c = a.c + g.vc, *lv = a.lv + g.vc, *uv = a.uv + g.vc;
        double *lc = a.lc + g.vr, *uc = a.uc + g.vr;
        double *x = a.x + g.vc, *x0 = a.x0 + g.vc, *xh = a.xh + g.vc, *xe = a.xe + g.vc;
        double *aty = a.aty + g.vc;
        double *y = a.y + g.vr, *y0 = a.y0 + g.vr, *yh = a.yh + g.vr;
        const double eta = a.eta[g.sidx];
        const double gam = o.gamma;

        // scaled data, norms, initial point
        double nrm[4] = {0.0, 0.0, 0.0, 0.0};
        for (int32_t j = threadIdx.x; j < g.n; j += BT) {
            const double d = Dc[j];
            const double cj = d * c_o[j];
            c[j] = cj;
            lv[j] = lv_o[j] / d;
            uv[j] = uv_o[j] / d;
            nrm[0] += cj * cj;
            nrm[2] += c_o[j] * c_o[j];
        }
        for (int32_t i = threadIdx.x; i < g.m; i += BT) {
            const double d = Dr[i];
            const double l = d * lc_o[i], u = d * uc_o[i];
            lc[i] = l;
            uc[i] = u;
            double bb = 0.0, bo = 0.0;
            if (isfinite(l)) bb = fmax(bb, fabs(l));
            if (isfinite(u)) bb = fmax(bb, fabs(u));
            if (isfinite(lc_o[i])) bo = fmax(bo, fabs(lc_o[i]));
            if (isfinite(uc_o[i])) bo = fmax(bo, fabs(uc_o[i]));
            nrm[1] += bb * bb;
            nrm[3] += bo * bo;
        }
        wg_sum<BT, 4>(nrm);
        const double cn = sqrt(nrm[0]), bn = sqrt(nrm[1]);
        const double cnorm = sqrt(nrm[2]), bnorm = sqrt(nrm[3]);
        double omega = (cn > 1e-10 && bn > 1e-10) ? cn / bn : 1.0;
        double tau = eta / omega, sigma = eta * omega;
        for (int32_t j = threadIdx.x; j < g.n; j += BT) {
            const double v0 = a.x_init ? a.x_init[g.vc + j] / Dc[j] : 0.0;
            const double xv = clampd(v0, lv[j], uv[j]);
            x[j] = xv;
            x0[j] = xv;
        }
        for (int32_t i = threadIdx.x; i < g.m; i += BT) {
            const double v0 = a.y_init ? a.y_init[g.vr + i] / Dr[i] : 0.0;
            const double lo = isfinite(uc[i]) ? -INFINITY : 0.0;
            const double hi = isfinite(lc[i]) ? INFINITY : 0.0;
            const double yv = clampd(v0, lo, hi);
            y[i] = yv;
            y0[i] = yv;
        }
        __syncthreads();

        int64_t t = 0, k = 0, restarts = 0;
        double r_start = 0.0, r_prev = 0.0;
        int32_t status = 0;
        bool anchor_valid = false;   // the anchor's products are stored (after a restart)
        double ray_scale = 0.0;
        double kkt = 0.0, rel_p = 0.0, rel_d = 0.0, rel_g = 0.0, P = 0.0, D = 0.0;
        for (;;) {
            const bool check = (t % o.check_every) == 0;
            const bool last = t + 1 >= o.limit;
            const bool keep = check || last;
            const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
            // primal step over the rows of A'
            for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                const double s = csr_dot(trp, tci, tva, j, y);
                const double xr = x[j];
                const double xhat = clampd(xr - tau * (c[j] - s), lv[j], uv[j]);
                xe[j] = 2.0 * xhat - xr;
                if (keep) {
                    xh[j] = xhat;
                    aty[j] = s;
                } else {
                    x[j] = ak * ((1.0 + gam) * xhat - gam * xr) + bk * x0[j];
                }
            }
            __syncthreads();
            // dual step over the rows of A
            for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                const double av = csr_dot(arp, aci, ava, i, xe);
                const double yr = y[i];
                const double yhat = dual_prox(yr, av, sigma, lc[i], uc[i]);
                if (keep)
                    yh[i] = yhat;
                else
                    y[i] = ak * ((1.0 + gam) * yhat - gam * yr) + bk * y0[i];
            }
            __syncthreads();
            if (!keep) {
                ++k;
                ++t;
                continue;
            }
            // check: KKT in the original space and the fixed-point residual
            double v[10];
#pragma unroll
            for (int q = 0; q < 10; ++q) v[q] = 0.0;
            for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                const double q = csr_dot(trp, tci, tva, j, yh);
                const double xhv = xh[j];
                const double dx = xhv - x[j];
                v[0] += dx * dx;
                v[1] += (q - aty[j]) * dx;
                const double d0 = xhv - x0[j];
                v[2] += d0 * d0;
                const double d = Dc[j];
                const double gr = c_o[j] - q / d;
                const double lo = lv_o[j], hi = uv_o[j];
                const bool lf = isfinite(lo), uf = isfinite(hi);
                const double lam = (!lf && !uf) ? 0.0 : (lf && !uf) ? fmax(gr, 0.0) : (!lf && uf) ? fmin(gr, 0.0) : gr;
                const double rd = gr - lam;
                v[3] += rd * rd;
                v[4] += c_o[j] * (d * xhv);
                v[5] += (lf ? lo * fmax(lam, 0.0) : 0.0) - (uf ? hi * fmax(-lam, 0.0) : 0.0);
                if (RAYS) a.qh[g.vc + j] = q;
            }
            for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                const double p = csr_dot(arp, aci, ava, i, xh);
                const double d = Dr[i];
                const double ax = p / d;
                const double lo = lc_o[i], hi = uc_o[i];
                const double rpr = ax - clampd(ax, lo, hi);
                v[6] += rpr * rpr;
                const double yhv = yh[i];
                const double yo = d * yhv;
                v[7] += (isfinite(lo) ? lo * fmax(yo, 0.0) : 0.0) - (isfinite(hi) ? hi * fmax(-yo, 0.0) : 0.0);
                const double dy = yhv - y[i];
                v[8] += dy * dy;
                const double d0 = yhv - y0[i];
                v[9] += d0 * d0;
                if (RAYS) a.ph[g.vr + i] = p;
            }
            wg_sum<BT, 10>(v);
            P = v[4];
            D = v[7] + v[5];
            rel_p = sqrt(v[6]) / (1.0 + bnorm);
            rel_d = sqrt(v[3]) / (1.0 + cnorm);
            rel_g = fabs(P - D) / (1.0 + fabs(P) + fabs(D));
            kkt = rel_p;
            if (rel_d > kkt || isnan(rel_d)) kkt = rel_d;
            if (rel_g > kkt || isnan(rel_g)) kkt = rel_g;
            if (isnan(kkt)) {
                status = PDHG_NUMERICAL_ERROR;
                break;
            }
            if (kkt <= o.eps) {
                status = PDHG_OPTIMAL;
                break;
            }
            if (RAYS && anchor_valid) {
                double rs[3], rm[2];
                batch_ray_pass<BT>(a, g, xh, yh, y0, rs, rm);
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
            if (last) {
                status = PDHG_ITERATION_LIMIT;
                break;
            }
            const double r2 = v[0] / tau + v[8] / sigma + 2.0 * v[1];
            const double r = r2 > 0.0 ? sqrt(r2) : 0.0;
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
                const double dxr = sqrt(v[2]), dyr = sqrt(v[9]);
                omega = batch_new_omega(omega, dxr, dyr);
                tau = eta / omega;
                sigma = eta * omega;
                for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                    x[j] = xh[j];
                    x0[j] = xh[j];
                }
                for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                    y[i] = yh[i];
                    y0[i] = yh[i];
                }
                if (RAYS) {   // the new anchor's products, from this check
                    int32_t t0 = (int32_t)threadIdx.x;
                    asm volatile("" : "+v"(t0));
                    for (int32_t j = t0; j < g.n; j += BT) a.q0[g.vc + j] = a.qh[g.vc + j];
                    for (int32_t i = t0; i < g.m; i += BT) a.p0[g.vr + i] = a.ph[g.vr + i];
                    anchor_valid = true;
                }
                k = 0;
                r_start = r;
                r_prev = r;
                ++restarts;
            } else {
                for (int32_t j = threadIdx.x; j < g.n; j += BT)
                    x[j] = ak * ((1.0 + gam) * xh[j] - gam * x[j]) + bk * x0[j];
                for (int32_t i = threadIdx.x; i < g.m; i += BT)
                    y[i] = ak * ((1.0 + gam) * yh[i] - gam * y[i]) + bk * y0[i];
                ++k;
            }
            ++t;
            __syncthreads();
        }
        // original-space output of the last PDHG point, or the certifying ray
        const bool xray = status == PDHG_DUAL_INFEASIBLE, yray = status == PDHG_PRIMAL_INFEASIBLE;
        for (int32_t j = threadIdx.x; j < g.n; j += BT)
            a.x_out[g.vc + j] = Dc[j] * (xray ? (xh[j] - x0[j]) * ray_scale : xh[j]);
        for (int32_t i = threadIdx.x; i < g.m; i += BT)
            a.y_out[g.vr + i] = Dr[i] * (yray ? (yh[i] - y0[i]) * ray_scale : yh[i]);
        if (threadIdx.x == 0) {
            BatchRes r;
            r.pobj = P;
            r.dobj = D;
            r.rel_p = rel_p;
            r.rel_d = rel_d;
            r.rel_g = rel_g;
            r.kkt = kkt;
            r.omega = omega;
            r.eta = eta;
            r.iterations = t + 1;
            r.restarts = restarts;
            r.status = status;
            r.power_iters = a.power_iters[g.sidx];
            a.res[b] = r;
        }
        __syncthreads();
    }
}

// Entries per column slice and per row slice of the register-resident matrix
// (node-arc incidence matrices: two entries per column, node degree <= 8).
constexpr int kResCol = 2, kResRow = 8;

// A double in LDS at a byte offset from the start of the dynamic allocation.
__device__ __forceinline__ double lds_at(const double *lds, int32_t off) {
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(lds) + off);
}

// Same iteration with the gathered vectors held on chip: y (for A~'y) and
// x_ext (for A~x_ext; at checks the PDHG points) live in LDS, next to the
// per-row anchor and bounds; each thread owns S columns and S rows (RES: S/4
// rows), in SELL-64 slices, so a wave's slices are whole.
//   RES = false: the matrix entries stream from the shared SELL-64 copies (L2)
//     on every product; the per-column iterate, anchor, cost and bounds stay
//     in registers.
//   RES = true (a shared matrix whose column slices hold at most kResCol and
//     row slices at most kResRow entries): every thread loads its slices'
//     entries once per instance into registers, with each index turned into
//     the byte offset of the LDS element it gathers, so an iteration reads no
//     matrix data from memory: a product is LDS gathers and FMAs. The anchor,
//     cost and upper bound of the columns move to LDS to make room.
// Entries past a slice's width are zeros gathering element 0, which adds
// +0 like the slices' own padding. Same arithmetic and summation order as
// k_batch_solve.
template <int BT, int S, bool RES, bool RAYS>
__global__ __launch_bounds__(BT) void k_batch_solve_lds(BArgs a, BOpts o, int32_t nmax, int32_t mmax) {
    constexpr int SR = RES ? (S >= 4 ? S / 4 : 1) : S;   // row slices per thread
    extern __shared__ double lds[];
    double *sx = lds;                 // x_ext, at checks x^
    double *sy = lds + nmax;          // y, at checks y^
    double *slc = sy + mmax;          // scaled row bounds
    double *suc = slc + mmax;
    double *y0 = suc + mmax;          // dual anchor
    double *sx0 = y0 + mmax;          // RES: primal anchor
    double *scr = sx0 + nmax;         // RES: scaled cost
    double *suv = scr + nmax;         // RES: scaled upper bound
    for (;;) {
        const int32_t b = next_instance<BT>(a.queue);
        if (b >= a.B) return;
        const Geo g = geometry(a, b);
        const int32_t as0 = a.shared ? 0 : a.asfirst[b], ts0 = a.shared ? 0 : a.tsfirst[b];
        const int32_t lane = (int32_t)(threadIdx.x & 63);
        const double *Dr = a.Dr + g.dr, *Dc = a.Dc + g.dc;
        const double *c_o = a.c_o + g.vc, *lv_o = a.lv_o + g.vc, *uv_o = a.uv_o + g.vc;
        const double *lc_o = a.lc_o + g.vr, *uc_o = a.uc_o + g.vr;
        double *__restrict__ xh = a.xh + g.vc;
        double *__restrict__ aty = a.aty + g.vc;
        double *__restrict__ y = a.y + g.vr;
        double *__restrict__ yh = a.yh + g.vr;
        const int32_t *__restrict__ tsci = a.tsci;
        const int32_t *__restrict__ asci = a.asci;
        const double *__restrict__ tsva = a.tsva;
        const double *__restrict__ asva = a.asva;
        const double eta = a.eta[g.sidx];
        const double gam = o.gamma;

        // streamed: slice start and width of each owned column / row
        int32_t tbase[S], tw[S], abase[S], aw[S];
        // resident: the owned slices' entries (LDS byte offset, value)
        int32_t tci[S][kResCol], rci[SR][kResRow];
        double tva[S][kResCol], rva[SR][kResRow];
        // per-column iterate and bounds in registers (streamed: also anchor, cost)
        double xr[S], x0r[S], cr[S], lvr[S], uvr[S];
        double nrm[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int32_t j = threadIdx.x + q * BT;
            tbase[q] = tw[q] = abase[q] = aw[q] = 0;
            xr[q] = x0r[q] = cr[q] = lvr[q] = uvr[q] = 0.0;
            if (j < g.n) {
                const int32_t sl = ts0 + (j >> 6);
                tbase[q] = a.tsp[sl];
                tw[q] = (a.tsp[sl + 1] - tbase[q]) >> 6;
            }
            if (q < SR && j < g.m) {
                const int32_t sl = as0 + (j >> 6);
                abase[q] = a.asp[sl];
                aw[q] = (a.asp[sl + 1] - abase[q]) >> 6;
            }
            if (j < g.n) {
                const double d = Dc[j];
                const double cj = d * c_o[j];
                const double l = lv_o[j] / d, u = uv_o[j] / d;
                if constexpr (RES) scr[j] = cj;
                else cr[q] = cj;
                lvr[q] = l;
                if constexpr (RES) suv[j] = u;
                else uvr[q] = u;
                nrm[0] += cj * cj;
                nrm[2] += c_o[j] * c_o[j];
                const double v0 = a.x_init ? a.x_init[g.vc + j] / d : 0.0;
                xr[q] = clampd(v0, l, u);
                if constexpr (RES) sx0[j] = xr[q];
                else x0r[q] = xr[q];
            }
            const int32_t i = j;
            if (q < SR && i < g.m) {
                const double d = Dr[i];
                const double l = d * lc_o[i], u = d * uc_o[i];
                slc[i] = l;
                suc[i] = u;
                double bb = 0.0, bo = 0.0;
                if (isfinite(l)) bb = fmax(bb, fabs(l));
                if (isfinite(u)) bb = fmax(bb, fabs(u));
                if (isfinite(lc_o[i])) bo = fmax(bo, fabs(lc_o[i]));
                if (isfinite(uc_o[i])) bo = fmax(bo, fabs(uc_o[i]));
                nrm[1] += bb * bb;
                nrm[3] += bo * bo;
                const double v0 = a.y_init ? a.y_init[g.vr + i] / d : 0.0;
                const double lo = isfinite(u) ? -INFINITY : 0.0;
                const double hi = isfinite(l) ? INFINITY : 0.0;
                const double yv = clampd(v0, lo, hi);
                sy[i] = yv;
                y0[i] = yv;
            }
        }
        // RES: the owned slices' entries into registers
        auto load_matrix = [&]() {
            if constexpr (RES) {
#pragma unroll
                for (int q = 0; q < S; ++q) {
#pragma unroll
                    for (int u = 0; u < kResCol; ++u) {
                        const bool in = u < tw[q];
                        const int32_t e = tbase[q] + 64 * u + lane;
                        tci[q][u] = 8 * (nmax + (in ? tsci[e] : 0));
                        tva[q][u] = in ? tsva[e] : 0.0;
                    }
                }
#pragma unroll
                for (int q = 0; q < SR; ++q) {
#pragma unroll
                    for (int u = 0; u < kResRow; ++u) {
                        const bool in = u < aw[q];
                        const int32_t e = abase[q] + 64 * u + lane;
                        rci[q][u] = 8 * (in ? asci[e] : 0);
                        rva[q][u] = in ? asva[e] : 0.0;
                    }
                }
            }
        };
        load_matrix();
        // A~'y (gathering y from LDS) for owned column q; A~x_ext for owned row q
        auto col_dot = [&](int q) -> double {
            if constexpr (RES) {
                double s = 0.0;
#pragma unroll
                for (int u = 0; u < kResCol; ++u) s = fma(tva[q][u], lds_at(lds, tci[q][u]), s);
                return s;
            } else {
                return sell_dot_bw(tsci, tsva, tbase[q], tw[q], lane, sy);
            }
        };
        auto row_dot = [&](int q) -> double {
            if constexpr (RES) {
                double s = 0.0;
#pragma unroll
                for (int u = 0; u < kResRow; ++u) s = fma(rva[q][u], lds_at(lds, rci[q][u]), s);
                return s;
            } else {
                return sell_dot_bw(asci, asva, abase[q], aw[q], lane, sx);
            }
        };
        auto x0_of = [&](int q, int32_t j) -> double {
            if constexpr (RES) return sx0[j];
            else return x0r[q];
        };
        auto set_x0 = [&](int q, int32_t j, double v) {
            if constexpr (RES) sx0[j] = v;
            else x0r[q] = v;
        };
        auto c_of = [&](int q, int32_t j) -> double {
            if constexpr (RES) return scr[j];
            else return cr[q];
        };
        auto uv_of = [&](int q, int32_t j) -> double {
            if constexpr (RES) return suv[j];
            else return uvr[q];
        };
        wg_sum<BT, 4>(nrm);
        const double cn = sqrt(nrm[0]), bn = sqrt(nrm[1]);
        const double cnorm = sqrt(nrm[2]), bnorm = sqrt(nrm[3]);
        double omega = (cn > 1e-10 && bn > 1e-10) ? cn / bn : 1.0;
        double tau = eta / omega, sigma = eta * omega;

        int64_t t = 0, k = 0, restarts = 0;
        int32_t tc = 0;   // t modulo check_every, without a 64-bit division per iteration
        double r_start = 0.0, r_prev = 0.0;
        int32_t status = 0;
        bool anchor_valid = false;   // the anchor's products are stored (after a restart)
        double ray_scale = 0.0;
        double kkt = 0.0, rel_p = 0.0, rel_d = 0.0, rel_g = 0.0, P = 0.0, D = 0.0;
        for (;;) {
            // an opaque copy of the thread index: the element addresses are
            // recomputed each iteration (two VALU ops) instead of being hoisted
            // into ~40 registers per slot, which would spill
            int32_t tid = (int32_t)threadIdx.x;
            asm volatile("" : "+v"(tid));
            const bool check = tc == 0;
            const bool last = t + 1 >= o.limit;
            const bool keep = check || last;
            const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int32_t j = tid + q * BT;
                if (j < g.n) {
                    const double s = col_dot(q);
                    const double xhat = clampd(xr[q] - tau * (c_of(q, j) - s), lvr[q], uv_of(q, j));
                    sx[j] = 2.0 * xhat - xr[q];
                    if (keep) {
                        xh[j] = xhat;
                        aty[j] = s;
                    } else {
                        xr[q] = ak * ((1.0 + gam) * xhat - gam * xr[q]) + bk * x0_of(q, j);
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < SR; ++q) {
                const int32_t i = tid + q * BT;
                if (i < g.m) {
                    const double av = row_dot(q);
                    const double li = slc[i], ui = suc[i];
                    const double yv = sy[i];
                    const double yhat = dual_prox(yv, av, sigma, li, ui);
                    if (keep) {
                        yh[i] = yhat;
                        y[i] = yv;
                    } else {
                        sy[i] = ak * ((1.0 + gam) * yhat - gam * yv) + bk * y0[i];
                    }
                }
            }
            __syncthreads();
            if (!keep) {
                ++k;
                ++t;
                tc = tc + 1 == o.check_every ? 0 : tc + 1;
                continue;
            }
            // check: the PDHG points replace x_ext and y in LDS for the products
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int32_t j = tid + q * BT;
                if (j < g.n) sx[j] = xh[j];
                if (q < SR && j < g.m) sy[j] = yh[j];
            }
            __syncthreads();
            // KKT sums, then (RAYS) the ray sums: v[10], v[11] over the columns
            // (bound terms, c'dx), v[12] over the rows; rmx the ray violations
            constexpr int NV = RAYS ? 13 : 10;
            double v[NV], rmx[2] = {0.0, 0.0};
#pragma unroll
            for (int q = 0; q < NV; ++q) v[q] = 0.0;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int32_t j = tid + q * BT;
                if (j < g.n) {
                    const double qq = col_dot(q);
                    const double xhv = xh[j];
                    const double dx = xhv - xr[q];
                    v[0] += dx * dx;
                    v[1] += (qq - aty[j]) * dx;
                    const double d0 = xhv - x0_of(q, j);
                    v[2] += d0 * d0;
                    const double d = Dc[j];
                    const double gr = c_o[j] - qq / d;
                    const double lo = lv_o[j], hi = uv_o[j];
                    const bool lf = isfinite(lo), uf = isfinite(hi);
                    const double lam = (!lf && !uf) ? 0.0 : (lf && !uf) ? fmax(gr, 0.0) : (!lf && uf) ? fmin(gr, 0.0) : gr;
                    const double rd = gr - lam;
                    v[3] += rd * rd;
                    v[4] += c_o[j] * (d * xhv);
                    v[5] += (lf ? lo * fmax(lam, 0.0) : 0.0) - (uf ? hi * fmax(-lam, 0.0) : 0.0);
                    if constexpr (RAYS) {
                        a.qh[g.vc + j] = qq;
                        double s2[2], m2[2];
                        ray_col_terms(qq, a.q0[g.vc + j], d, xhv - x0_of(q, j), c_o[j], lo, hi, s2, m2);
                        v[10] += s2[0];
                        v[11] += s2[1];
                        rmx[0] = fmax(rmx[0], m2[0]);
                        rmx[1] = fmax(rmx[1], m2[1]);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < SR; ++q) {
                const int32_t i = tid + q * BT;
                if (i < g.m) {
                    const double p = row_dot(q);
                    const double d = Dr[i];
                    const double ax = p / d;
                    const double lo = lc_o[i], hi = uc_o[i];
                    const double rpr = ax - clampd(ax, lo, hi);
                    v[6] += rpr * rpr;
                    const double yhv = yh[i];
                    const double yo = d * yhv;
                    v[7] += (isfinite(lo) ? lo * fmax(yo, 0.0) : 0.0) - (isfinite(hi) ? hi * fmax(-yo, 0.0) : 0.0);
                    const double dy = yhv - y[i];
                    v[8] += dy * dy;
                    const double d0 = yhv - y0[i];
                    v[9] += d0 * d0;
                    if constexpr (RAYS) {
                        a.ph[g.vr + i] = p;
                        double s1[1], m2[2];
                        ray_row_terms(p, a.p0[g.vr + i], d, d0, lo, hi, s1, m2);
                        v[12] += s1[0];
                        rmx[0] = fmax(rmx[0], m2[0]);
                        rmx[1] = fmax(rmx[1], m2[1]);
                    }
                }
            }
            wg_sum<BT, NV>(v);
            P = v[4];
            D = v[7] + v[5];
            rel_p = sqrt(v[6]) / (1.0 + bnorm);
            rel_d = sqrt(v[3]) / (1.0 + cnorm);
            rel_g = fabs(P - D) / (1.0 + fabs(P) + fabs(D));
            kkt = rel_p;
            if (rel_d > kkt || isnan(rel_d)) kkt = rel_d;
            if (rel_g > kkt || isnan(rel_g)) kkt = rel_g;
            if (isnan(kkt)) {
                status = PDHG_NUMERICAL_ERROR;
                break;
            }
            if (kkt <= o.eps) {
                status = PDHG_OPTIMAL;
                break;
            }
            if (RAYS && anchor_valid) {
                // the rays' terms were summed in the check loops above, in
                // the order of the separate pass of k_batch_solve
                double rs[3] = {v[RAYS ? 10 : 0], v[RAYS ? 11 : 0], v[RAYS ? 12 : 0]};
                double rm[2] = {rmx[0], rmx[1]};
                wg_max<BT, 2>(rm);
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
            if (last) {
                status = PDHG_ITERATION_LIMIT;
                break;
            }
            const double r2 = v[0] / tau + v[8] / sigma + 2.0 * v[1];
            const double r = r2 > 0.0 ? sqrt(r2) : 0.0;
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
                const double dxr = sqrt(v[2]), dyr = sqrt(v[9]);
                omega = batch_new_omega(omega, dxr, dyr);
                tau = eta / omega;
                sigma = eta * omega;
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    const int32_t j = tid + q * BT;
                    if (j < g.n) {
                        xr[q] = xh[j];
                        set_x0(q, j, xr[q]);
                    }
                    if (q < SR && j < g.m) {
                        sy[j] = yh[j];
                        y0[j] = yh[j];
                    }
                }
                if (RAYS) {   // the new anchor's products, from this check
                    int32_t t0 = (int32_t)threadIdx.x;
                    asm volatile("" : "+v"(t0));
                    for (int32_t j = t0; j < g.n; j += BT) a.q0[g.vc + j] = a.qh[g.vc + j];
                    for (int32_t i = t0; i < g.m; i += BT) a.p0[g.vr + i] = a.ph[g.vr + i];
                    anchor_valid = true;
                }
                k = 0;
                r_start = r;
                r_prev = r;
                ++restarts;
            } else {
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    const int32_t j = tid + q * BT;
                    if (j < g.n) xr[q] = ak * ((1.0 + gam) * xh[j] - gam * xr[q]) + bk * x0_of(q, j);
                    if (q < SR && j < g.m) sy[j] = ak * ((1.0 + gam) * yh[j] - gam * y[j]) + bk * y0[j];
                }
                ++k;
            }
            ++t;
            tc = tc + 1 == o.check_every ? 0 : tc + 1;
            __syncthreads();
        }
        // original-space output of the last PDHG point, or the certifying ray
        const bool xray = status == PDHG_DUAL_INFEASIBLE, yray = status == PDHG_PRIMAL_INFEASIBLE;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int32_t j = threadIdx.x + q * BT;
            if (j < g.n) a.x_out[g.vc + j] = Dc[j] * (xray ? (xh[j] - x0_of(q, j)) * ray_scale : xh[j]);
            if (q < SR && j < g.m) a.y_out[g.vr + j] = Dr[j] * (yray ? (yh[j] - y0[j]) * ray_scale : yh[j]);
        }
        if (threadIdx.x == 0) {
            BatchRes r;
            r.pobj = P;
            r.dobj = D;
            r.rel_p = rel_p;
            r.rel_d = rel_d;
            r.rel_g = rel_g;
            r.kkt = kkt;
            r.omega = omega;
            r.eta = eta;
            r.iterations = t + 1;
            r.restarts = restarts;
            r.status = status;
            r.power_iters = a.power_iters[g.sidx];
            a.res[b] = r;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// unrolled iterations with a frozen schedule, and their reverse pass

struct UArgs {
    int64_t T;
    int32_t replay;                       // 1: take restarts / weights from the schedule
    uint8_t *restart;                     // [B][T]
    double *omega;                        // [B][T]
    int32_t *kk;                          // [B][T]
    uint64_t *xmask, *ymask;              // bit-packed projection states
    const int64_t *xm_off, *ym_off;       // per-instance word offsets
    const double *gx, *gy;                // cotangents of the outputs
    double *gc, *glc, *guc;               // gradients (original space)
    double *ba;                           // scratch, like lc
};

// Exactly T iterations of Algorithm 1 per instance. Restart tests run at the
// check cadence (no termination test) unless replayed; every iteration
// records omega, k, the restart flag, the set of x inside its box and the
// clamp state of every row (bit 0: at -u_c, bit 1: at -l_c).
// ONCHIP: y and x_ext live in LDS and the products walk the SELL-64 copies
// (instances whose n + m fits the LDS budget); otherwise everything stays in
// memory and the products walk the CSR arrays. Same arithmetic either way.
template <int BT, bool ONCHIP>
__global__ __launch_bounds__(BT) void k_batch_unrolled(BArgs a, BOpts o, UArgs u, int32_t nmax) {
    extern __shared__ double lds[];
    for (;;) {
        const int32_t b = next_instance<BT>(a.queue);
        if (b >= a.B) return;
        const Geo g = geometry(a, b);
        const int32_t *arp = a.arp + g.r0, *trp = a.trp + g.c0;
        const int32_t *aci = a.aci, *tci = a.tci;
        const double *ava = a.ava, *tva = a.tva;
        const double *Dr = a.Dr + g.dr, *Dc = a.Dc + g.dc;
        const double *c_o = a.c_o + g.vc, *lv_o = a.lv_o + g.vc, *uv_o = a.uv_o + g.vc;
        const double *lc_o = a.lc_o + g.vr, *uc_o = a.uc_o + g.vr;
        double *c = a.c + g.vc, *lv = a.lv + g.vc, *uv = a.uv + g.vc;
        double *lc = a.lc + g.vr, *uc = a.uc + g.vr;
        double *x = a.x + g.vc, *x0 = a.x0 + g.vc, *xh = a.xh + g.vc, *xe = a.xe + g.vc;
        double *aty = a.aty + g.vc;
        double *y0 = a.y0 + g.vr, *yh = a.yh + g.vr;
        // gathered vectors: y (primal product) and x_ext (dual product)
        double *y = ONCHIP ? lds + nmax : a.y + g.vr;
        if (ONCHIP) xe = lds;
        const int32_t as0 = (ONCHIP && !a.shared) ? a.asfirst[b] : 0;
        const int32_t ts0 = (ONCHIP && !a.shared) ? a.tsfirst[b] : 0;
        uint8_t *rs_ = u.restart + (size_t)b * u.T;
        double *om_ = u.omega + (size_t)b * u.T;
        int32_t *kk_ = u.kk + (size_t)b * u.T;
        uint64_t *xm = u.xmask + u.xm_off[b], *ym = u.ymask + u.ym_off[b];
        const int32_t xw = (g.n + 63) >> 6, yw = (g.m + 63) >> 6;
        const double eta = a.eta[g.sidx];
        const double gam = o.gamma;
        double nrm[2] = {0.0, 0.0};
        for (int32_t j = threadIdx.x; j < g.n; j += BT) {
            const double d = Dc[j];
            const double cj = d * c_o[j];
            c[j] = cj;
            lv[j] = lv_o[j] / d;
            uv[j] = uv_o[j] / d;
            nrm[0] += cj * cj;
        }
        for (int32_t i = threadIdx.x; i < g.m; i += BT) {
            const double d = Dr[i];
            const double l = d * lc_o[i], uu = d * uc_o[i];
            lc[i] = l;
            uc[i] = uu;
            double bb = 0.0;
            if (isfinite(l)) bb = fmax(bb, fabs(l));
            if (isfinite(uu)) bb = fmax(bb, fabs(uu));
            nrm[1] += bb * bb;
        }
        wg_sum<BT, 2>(nrm);
        const double cn = sqrt(nrm[0]), bn = sqrt(nrm[1]);
        double omega = (cn > 1e-10 && bn > 1e-10) ? cn / bn : 1.0;
        for (int32_t j = threadIdx.x; j < g.n; j += BT) {
            const double xv = clampd(0.0, lv[j], uv[j]);
            x[j] = xv;
            x0[j] = xv;
        }
        for (int32_t i = threadIdx.x; i < g.m; i += BT) {
            const double lo = isfinite(uc[i]) ? -INFINITY : 0.0;
            const double hi = isfinite(lc[i]) ? INFINITY : 0.0;
            const double yv = clampd(0.0, lo, hi);
            y[i] = yv;
            y0[i] = yv;
        }
        __syncthreads();
        int64_t k = 0;
        double r_start = 0.0, r_prev = 0.0;
        for (int64_t t = 0; t < u.T; ++t) {
            if (u.replay) omega = om_[t];
            const double tau = eta / omega, sigma = eta * omega;
            const bool last = t + 1 >= u.T;
            const bool check = !u.replay && (t % o.check_every) == 0 && !last;
            const bool keep = true;   // restart decisions need the PDHG point
            const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
            (void)keep;
            uint64_t *xmt = xm + (size_t)t * xw;
            uint64_t *ymt = ym + (size_t)t * 2 * yw;
            for (int32_t j0 = 0; j0 < g.n; j0 += BT) {
                const int32_t j = j0 + (int32_t)threadIdx.x;
                bool inside = false;
                if (j < g.n) {
                    const double s = ONCHIP ? sell_dot(a.tsp, a.tsci, a.tsva, ts0 + (j >> 6), j & 63, y)
                                            : csr_dot(trp, tci, tva, j, y);
                    const double xr = x[j];
                    const double uu = xr - tau * (c[j] - s);
                    inside = uu > lv[j] && uu < uv[j];
                    const double xhat = clampd(uu, lv[j], uv[j]);
                    xe[j] = 2.0 * xhat - xr;
                    xh[j] = xhat;
                    aty[j] = s;
                }
                const uint64_t bits = __ballot(inside);
                if ((threadIdx.x & 63) == 0 && j < g.n) xmt[j >> 6] = bits;
            }
            __syncthreads();
            for (int32_t i0 = 0; i0 < g.m; i0 += BT) {
                const int32_t i = i0 + (int32_t)threadIdx.x;
                bool at_u = false, at_l = false;
                if (i < g.m) {
                    const double av = ONCHIP ? sell_dot(a.asp, a.asci, a.asva, as0 + (i >> 6), i & 63, xe)
                                             : csr_dot(arp, aci, ava, i, xe);
                    const double vv = y[i] / sigma - av;
                    at_u = vv < -uc[i];
                    at_l = vv > -lc[i];
                    yh[i] = sigma * (vv - clampd(vv, -uc[i], -lc[i]));
                }
                const uint64_t bu = __ballot(at_u), bl = __ballot(at_l);
                if ((threadIdx.x & 63) == 0 && i < g.m) {
                    ymt[2 * (i >> 6)] = bu;
                    ymt[2 * (i >> 6) + 1] = bl;
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                om_[t] = omega;
                kk_[t] = (int32_t)k;
            }
            if (last) break;
            bool restart = u.replay ? rs_[t] != 0 : false;
            double v2[10];
            if (check) {
#pragma unroll
                for (int q = 0; q < 10; ++q) v2[q] = 0.0;
                for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                    const double dx = xh[j] - x[j];
                    v2[0] += dx * dx;
                    const double d0 = xh[j] - x0[j];
                    v2[2] += d0 * d0;
                    if (ONCHIP) xe[j] = dx;   // x_ext is spent: it carries dx for the cross term
                }
                if (ONCHIP) __syncthreads();
                for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                    const double dy = yh[i] - y[i];
                    v2[8] += dy * dy;
                    const double d0 = yh[i] - y0[i];
                    v2[9] += d0 * d0;
                    // cross term dy' A~ dx
                    double adx = 0.0;
                    if (ONCHIP) {
                        adx = sell_dot(a.asp, a.asci, a.asva, as0 + (i >> 6), i & 63, xe);
                    } else {
                        for (int32_t e = arp[i]; e < arp[i + 1]; ++e)
                            adx = fma(ava[e], xh[aci[e]] - x[aci[e]], adx);
                    }
                    v2[1] += dy * adx;
                }
                wg_sum<BT, 10>(v2);
                const double r2 = v2[0] / tau + v2[8] / sigma + 2.0 * v2[1];
                const double r = r2 > 0.0 ? sqrt(r2) : 0.0;
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
                    const double dxr = sqrt(v2[2]), dyr = sqrt(v2[9]);
                    omega = batch_new_omega(omega, dxr, dyr);
                    r_start = r;
                    r_prev = r;
                }
            }
            if (threadIdx.x == 0 && !u.replay) rs_[t] = restart ? 1 : 0;
            if (restart) {
                for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                    x[j] = xh[j];
                    x0[j] = xh[j];
                }
                for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                    y[i] = yh[i];
                    y0[i] = yh[i];
                }
                k = 0;
            } else {
                for (int32_t j = threadIdx.x; j < g.n; j += BT)
                    x[j] = ak * ((1.0 + gam) * xh[j] - gam * x[j]) + bk * x0[j];
                for (int32_t i = threadIdx.x; i < g.m; i += BT)
                    y[i] = ak * ((1.0 + gam) * yh[i] - gam * y[i]) + bk * y0[i];
                ++k;
            }
            __syncthreads();
        }
        if (u.replay == 0 && threadIdx.x == 0) rs_[u.T - 1] = 0;
        for (int32_t j = threadIdx.x; j < g.n; j += BT) a.x_out[g.vc + j] = Dc[j] * xh[j];
        for (int32_t i = threadIdx.x; i < g.m; i += BT) a.y_out[g.vr + i] = Dr[i] * yh[i];
        __syncthreads();
    }
}

// Register-resident matrix for the unrolled forward and its reverse pass
// (a shared matrix whose column slices hold at most kResCol and row slices at
// most kResRow entries; S columns and S/4 rows per thread): the owned slices'
// entries with every index turned into the byte offset of the LDS element it
// gathers, y (for A~') after nmax doubles of x_ext (for A~).
template <int BT, int S>
struct ResSlices {
    static constexpr int SR = S >= 4 ? S / 4 : 1;
    int32_t tci[S][kResCol], rci[SR][kResRow];
    double tva[S][kResCol], rva[SR][kResRow];

    __device__ __forceinline__ void load(const BArgs &a, const Geo &g, int32_t nmax) {
        const int32_t lane = (int32_t)(threadIdx.x & 63);
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int32_t j = threadIdx.x + q * BT;
            int32_t base = 0, w = 0;
            if (j < g.n) {
                base = a.tsp[j >> 6];
                w = (a.tsp[(j >> 6) + 1] - base) >> 6;
            }
#pragma unroll
            for (int u = 0; u < kResCol; ++u) {
                const bool in = u < w;
                const int32_t e = base + 64 * u + lane;
                tci[q][u] = 8 * (nmax + (in ? a.tsci[e] : 0));
                tva[q][u] = in ? a.tsva[e] : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < SR; ++q) {
            const int32_t i = threadIdx.x + q * BT;
            int32_t base = 0, w = 0;
            if (i < g.m) {
                base = a.asp[i >> 6];
                w = (a.asp[(i >> 6) + 1] - base) >> 6;
            }
#pragma unroll
            for (int u = 0; u < kResRow; ++u) {
                const bool in = u < w;
                const int32_t e = base + 64 * u + lane;
                rci[q][u] = 8 * (in ? a.asci[e] : 0);
                rva[q][u] = in ? a.asva[e] : 0.0;
            }
        }
    }
    // (A~' y)_j of owned column q, y in LDS after nmax doubles
    __device__ __forceinline__ double col(const double *lds, int q) const {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < kResCol; ++u) s = fma(tva[q][u], lds_at(lds, tci[q][u]), s);
        return s;
    }
    // (A~ v)_i of owned row q, v at the start of the LDS
    __device__ __forceinline__ double row(const double *lds, int q) const {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < kResRow; ++u) s = fma(rva[q][u], lds_at(lds, rci[q][u]), s);
        return s;
    }
};

// k_batch_unrolled for a register-resident shared matrix (grid batches): the
// same iterations, records and arithmetic, with x, x^ and l~_v of the owned
// columns and y^ of the owned rows in registers, and x_ext, y, x0, y0, c~,
// u~_v, l~_c, u~_c in LDS.
template <int BT, int S>
__global__ __launch_bounds__(BT) void k_batch_unrolled_res(BArgs a, BOpts o, UArgs u, int32_t nmax,
                                                           int32_t mmax) {
    using RS = ResSlices<BT, S>;
    constexpr int SR = RS::SR;
    extern __shared__ double lds[];
    double *sx = lds, *sy = lds + nmax;
    double *slc = sy + mmax, *suc = slc + mmax, *sy0 = suc + mmax;
    double *sx0 = sy0 + mmax, *scr = sx0 + nmax, *suv = scr + nmax;
    for (;;) {
        const int32_t b = next_instance<BT>(a.queue);
        if (b >= a.B) return;
        const Geo g = geometry(a, b);
        const int32_t lane = (int32_t)(threadIdx.x & 63);
        const double *Dr = a.Dr + g.dr, *Dc = a.Dc + g.dc;
        const double *c_o = a.c_o + g.vc, *lv_o = a.lv_o + g.vc, *uv_o = a.uv_o + g.vc;
        const double *lc_o = a.lc_o + g.vr, *uc_o = a.uc_o + g.vr;
        uint8_t *rs_ = u.restart + (size_t)b * u.T;
        double *om_ = u.omega + (size_t)b * u.T;
        int32_t *kk_ = u.kk + (size_t)b * u.T;
        uint64_t *xm = u.xmask + u.xm_off[b], *ym = u.ymask + u.ym_off[b];
        const int32_t xw = (g.n + 63) >> 6, yw = (g.m + 63) >> 6;
        const double eta = a.eta[g.sidx];
        const double gam = o.gamma;
        RS M;
        M.load(a, g, nmax);
        double xr[S], xhr[S], lvr[S], yhr[SR];
        double nrm[2] = {0.0, 0.0};
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int32_t j = threadIdx.x + q * BT;
            xr[q] = xhr[q] = lvr[q] = 0.0;
            if (j < g.n) {
                const double d = Dc[j];
                const double cj = d * c_o[j];
                scr[j] = cj;
                lvr[q] = lv_o[j] / d;
                suv[j] = uv_o[j] / d;
                nrm[0] += cj * cj;
            }
        }
#pragma unroll
        for (int q = 0; q < SR; ++q) {
            const int32_t i = threadIdx.x + q * BT;
            yhr[q] = 0.0;
            if (i < g.m) {
                const double d = Dr[i];
                const double l = d * lc_o[i], uu = d * uc_o[i];
                slc[i] = l;
                suc[i] = uu;
                double bb = 0.0;
                if (isfinite(l)) bb = fmax(bb, fabs(l));
                if (isfinite(uu)) bb = fmax(bb, fabs(uu));
                nrm[1] += bb * bb;
            }
        }
        wg_sum<BT, 2>(nrm);
        const double cn = sqrt(nrm[0]), bn = sqrt(nrm[1]);
        double omega = (cn > 1e-10 && bn > 1e-10) ? cn / bn : 1.0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int32_t j = threadIdx.x + q * BT;
            if (j < g.n) {
                xr[q] = clampd(0.0, lvr[q], suv[j]);
                sx0[j] = xr[q];
            }
        }
#pragma unroll
        for (int q = 0; q < SR; ++q) {
            const int32_t i = threadIdx.x + q * BT;
            if (i < g.m) {
                const double lo = isfinite(suc[i]) ? -INFINITY : 0.0;
                const double hi = isfinite(slc[i]) ? INFINITY : 0.0;
                const double yv = clampd(0.0, lo, hi);
                sy[i] = yv;
                sy0[i] = yv;
            }
        }
        __syncthreads();
        int64_t k = 0;
        int32_t tc = 0;   // t modulo check_every
        double r_start = 0.0, r_prev = 0.0;
        for (int64_t t = 0; t < u.T; ++t) {
            // opaque thread index: element addresses are formed per iteration
            int32_t tid = (int32_t)threadIdx.x;
            asm volatile("" : "+v"(tid));
            if (u.replay) omega = om_[t];
            const double tau = eta / omega, sigma = eta * omega;
            const bool last = t + 1 >= u.T;
            const bool check = !u.replay && tc == 0 && !last;
            const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
            uint64_t *xmt = xm + (size_t)t * xw;
            uint64_t *ymt = ym + (size_t)t * 2 * yw;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int32_t j = tid + q * BT;
                bool inside = false;
                if (j < g.n) {
                    const double s = M.col(lds, q);
                    const double uu = xr[q] - tau * (scr[j] - s);
                    const double hi = suv[j];
                    inside = uu > lvr[q] && uu < hi;
                    const double xhat = clampd(uu, lvr[q], hi);
                    sx[j] = 2.0 * xhat - xr[q];
                    xhr[q] = xhat;
                }
                const uint64_t bits = __ballot(inside);
                if (lane == 0 && j < g.n) xmt[j >> 6] = bits;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < SR; ++q) {
                const int32_t i = tid + q * BT;
                bool at_u = false, at_l = false;
                if (i < g.m) {
                    const double av = M.row(lds, q);
                    const double vv = sy[i] / sigma - av;
                    const double lo = -suc[i], hi = -slc[i];
                    at_u = vv < lo;
                    at_l = vv > hi;
                    yhr[q] = sigma * (vv - clampd(vv, lo, hi));
                }
                const uint64_t bu = __ballot(at_u), bl = __ballot(at_l);
                if (lane == 0 && i < g.m) {
                    ymt[2 * (i >> 6)] = bu;
                    ymt[2 * (i >> 6) + 1] = bl;
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                om_[t] = omega;
                kk_[t] = (int32_t)k;
            }
            if (last) break;
            bool restart = u.replay ? rs_[t] != 0 : false;
            if (check) {
                double v2[10];
#pragma unroll
                for (int q = 0; q < 10; ++q) v2[q] = 0.0;
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    const int32_t j = tid + q * BT;
                    if (j < g.n) {
                        const double dx = xhr[q] - xr[q];
                        v2[0] += dx * dx;
                        const double d0 = xhr[q] - sx0[j];
                        v2[2] += d0 * d0;
                        sx[j] = dx;   // x_ext is spent: it carries dx for the cross term
                    }
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < SR; ++q) {
                    const int32_t i = tid + q * BT;
                    if (i < g.m) {
                        const double dy = yhr[q] - sy[i];
                        v2[8] += dy * dy;
                        const double d0 = yhr[q] - sy0[i];
                        v2[9] += d0 * d0;
                        v2[1] += dy * M.row(lds, q);   // cross term dy' A~ dx
                    }
                }
                wg_sum<BT, 10>(v2);
                const double r2 = v2[0] / tau + v2[8] / sigma + 2.0 * v2[1];
                const double r = r2 > 0.0 ? sqrt(r2) : 0.0;
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
                    const double dxr = sqrt(v2[2]), dyr = sqrt(v2[9]);
                    omega = batch_new_omega(omega, dxr, dyr);
                    r_start = r;
                    r_prev = r;
                }
            }
            if (threadIdx.x == 0 && !u.replay) rs_[t] = restart ? 1 : 0;
            if (restart) {
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    const int32_t j = tid + q * BT;
                    if (j < g.n) {
                        xr[q] = xhr[q];
                        sx0[j] = xhr[q];
                    }
                }
#pragma unroll
                for (int q = 0; q < SR; ++q) {
                    const int32_t i = tid + q * BT;
                    if (i < g.m) {
                        sy[i] = yhr[q];
                        sy0[i] = yhr[q];
                    }
                }
                k = 0;
            } else {
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    const int32_t j = tid + q * BT;
                    if (j < g.n) xr[q] = ak * ((1.0 + gam) * xhr[q] - gam * xr[q]) + bk * sx0[j];
                }
#pragma unroll
                for (int q = 0; q < SR; ++q) {
                    const int32_t i = tid + q * BT;
                    if (i < g.m) sy[i] = ak * ((1.0 + gam) * yhr[q] - gam * sy[i]) + bk * sy0[i];
                }
                ++k;
            }
            tc = tc + 1 == o.check_every ? 0 : tc + 1;
            __syncthreads();
        }
        if (u.replay == 0 && threadIdx.x == 0) rs_[u.T - 1] = 0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int32_t j = threadIdx.x + q * BT;
            if (j < g.n) a.x_out[g.vc + j] = Dc[j] * xhr[q];
        }
#pragma unroll
        for (int q = 0; q < SR; ++q) {
            const int32_t i = threadIdx.x + q * BT;
            if (i < g.m) a.y_out[g.vr + i] = Dr[i] * yhr[q];
        }
        __syncthreads();
    }
}

// k_batch_backward for a register-resident shared matrix: the cotangents of
// the owned columns and rows and the gradient sums in registers; the products
// gather ba (after nmax doubles) and tmp (at the start) from LDS.
template <int BT, int S>
__global__ __launch_bounds__(BT) void k_batch_backward_res(BArgs a, BOpts o, UArgs u, int32_t nmax) {
    using RS = ResSlices<BT, S>;
    constexpr int SR = RS::SR;
    extern __shared__ double lds[];
    double *tmp = lds, *ba = lds + nmax;
    for (;;) {
        const int32_t b = next_instance<BT>(a.queue);
        if (b >= a.B) return;
        const Geo g = geometry(a, b);
        const int32_t lane = (int32_t)(threadIdx.x & 63);
        const double *Dr = a.Dr + g.dr, *Dc = a.Dc + g.dc;
        const uint8_t *rs_ = u.restart + (size_t)b * u.T;
        const double *om_ = u.omega + (size_t)b * u.T;
        const int32_t *kk_ = u.kk + (size_t)b * u.T;
        const uint64_t *xm = u.xmask + u.xm_off[b], *ym = u.ymask + u.ym_off[b];
        const int32_t xw = (g.n + 63) >> 6, yw = (g.m + 63) >> 6;
        const double eta = a.eta[g.sidx];
        const double gam = o.gamma;
        RS M;
        M.load(a, g, nmax);
        double bx[S], bx0[S], bxh[S], gcr[S];
        double by[SR], by0[SR], byh[SR], glr[SR], gur[SR];
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int32_t j = threadIdx.x + q * BT;
            bx[q] = bx0[q] = gcr[q] = 0.0;
            bxh[q] = j < g.n ? Dc[j] * u.gx[g.vc + j] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < SR; ++q) {
            const int32_t i = threadIdx.x + q * BT;
            by[q] = by0[q] = glr[q] = gur[q] = 0.0;
            byh[q] = i < g.m ? Dr[i] * u.gy[g.vr + i] : 0.0;
        }
        for (int64_t t = u.T - 1; t >= 0; --t) {
            int32_t tid = (int32_t)threadIdx.x;
            asm volatile("" : "+v"(tid));
            const double omega = om_[t];
            const double tau = eta / omega, sigma = eta * omega;
            if (t < u.T - 1) {
                if (rs_[t]) {
#pragma unroll
                    for (int q = 0; q < S; ++q) {
                        bxh[q] = bx[q] + bx0[q];
                        bx[q] = 0.0;
                        bx0[q] = 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < SR; ++q) {
                        byh[q] = by[q] + by0[q];
                        by[q] = 0.0;
                        by0[q] = 0.0;
                    }
                } else {
                    const int64_t k = kk_[t];
                    const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
#pragma unroll
                    for (int q = 0; q < S; ++q) {
                        const double v = bx[q];
                        bxh[q] = ak * (1.0 + gam) * v;
                        bx0[q] += bk * v;
                        bx[q] = -ak * gam * v;
                    }
#pragma unroll
                    for (int q = 0; q < SR; ++q) {
                        const double v = by[q];
                        byh[q] = ak * (1.0 + gam) * v;
                        by0[q] += bk * v;
                        by[q] = -ak * gam * v;
                    }
                }
            }
            // dual step: yhat = sigma (v - clamp(v, -u_c, -l_c)), v = y/sigma - A~ xext
            const uint64_t *ymt = ym + (size_t)t * 2 * yw;
#pragma unroll
            for (int q = 0; q < SR; ++q) {
                const int32_t i = tid + q * BT;
                if (i < g.m) {
                    const uint64_t bit = 1ull << (i & 63);
                    const bool at_u = (ymt[2 * (i >> 6)] & bit) != 0;
                    const bool at_l = (ymt[2 * (i >> 6) + 1] & bit) != 0;
                    const double bv = (at_u || at_l) ? sigma * byh[q] : 0.0;
                    if (at_u) gur[q] += sigma * byh[q];
                    if (at_l) glr[q] += sigma * byh[q];
                    by[q] += bv / sigma;
                    ba[i] = -bv;
                }
            }
            __syncthreads();
            // xext = 2 xhat - x, then the primal step xhat = clamp(x - tau (c - A~'y))
            const uint64_t *xmt = xm + (size_t)t * xw;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int32_t j = tid + q * BT;
                if (j < g.n) {
                    const double bxe = M.col(lds, q);
                    const double bh = bxh[q] + 2.0 * bxe;
                    bx[q] -= bxe;
                    const bool inside = (xmt[j >> 6] >> (j & 63)) & 1ull;
                    const double bu = inside ? bh : 0.0;
                    bx[q] += bu;
                    gcr[q] += -tau * bu;
                    tmp[j] = tau * bu;
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < SR; ++q) {
                const int32_t i = tid + q * BT;
                if (i < g.m) by[q] += M.row(lds, q);
            }
            __syncthreads();
        }
        // c~ = D_c c, l~_c = D_r l_c, u~_c = D_r u_c
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int32_t j = threadIdx.x + q * BT;
            if (j < g.n) u.gc[g.vc + j] = Dc[j] * gcr[q];
        }
#pragma unroll
        for (int q = 0; q < SR; ++q) {
            const int32_t i = threadIdx.x + q * BT;
            if (i < g.m) {
                u.glc[g.vr + i] = isfinite(a.lc_o[g.vr + i]) ? Dr[i] * glr[q] : 0.0;
                u.guc[g.vr + i] = isfinite(a.uc_o[g.vr + i]) ? Dr[i] * gur[q] : 0.0;
            }
        }
        (void)lane;
        __syncthreads();
    }
}

// Reverse pass of k_batch_unrolled with its recorded schedule and masks.
template <int BT, bool ONCHIP>
__global__ __launch_bounds__(BT) void k_batch_backward(BArgs a, BOpts o, UArgs u, int32_t nmax) {
    extern __shared__ double lds[];
    for (;;) {
        const int32_t b = next_instance<BT>(a.queue);
        if (b >= a.B) return;
        const Geo g = geometry(a, b);
        const int32_t *arp = a.arp + g.r0, *trp = a.trp + g.c0;
        const int32_t *aci = a.aci, *tci = a.tci;
        const double *ava = a.ava, *tva = a.tva;
        const double *Dr = a.Dr + g.dr, *Dc = a.Dc + g.dc;
        const uint8_t *rs_ = u.restart + (size_t)b * u.T;
        const double *om_ = u.omega + (size_t)b * u.T;
        const int32_t *kk_ = u.kk + (size_t)b * u.T;
        const uint64_t *xm = u.xmask + u.xm_off[b], *ym = u.ymask + u.ym_off[b];
        const int32_t xw = (g.n + 63) >> 6, yw = (g.m + 63) >> 6;
        const double eta = a.eta[g.sidx];
        const double gam = o.gamma;
        // cotangents: bx, bx0, bxh (x, x0, xh), tmp (xe); by, by0, byh (y, y0, yh), ba
        double *bx = a.x + g.vc, *bx0 = a.x0 + g.vc, *bxh = a.xh + g.vc, *tmp = a.xe + g.vc;
        double *by = a.y + g.vr, *by0 = a.y0 + g.vr, *byh = a.yh + g.vr, *ba = u.ba + g.vr;
        // gathered vectors: ba (A~' ba) and tmp (A~ tmp)
        if (ONCHIP) {
            tmp = lds;
            ba = lds + nmax;
        }
        const int32_t as0 = (ONCHIP && !a.shared) ? a.asfirst[b] : 0;
        const int32_t ts0 = (ONCHIP && !a.shared) ? a.tsfirst[b] : 0;
        double *gc = u.gc + g.vc, *glc = u.glc + g.vr, *guc = u.guc + g.vr;
        for (int32_t j = threadIdx.x; j < g.n; j += BT) {
            bx[j] = 0.0;
            bx0[j] = 0.0;
            bxh[j] = Dc[j] * u.gx[g.vc + j];
            gc[j] = 0.0;
        }
        for (int32_t i = threadIdx.x; i < g.m; i += BT) {
            by[i] = 0.0;
            by0[i] = 0.0;
            byh[i] = Dr[i] * u.gy[g.vr + i];
            glc[i] = 0.0;
            guc[i] = 0.0;
        }
        __syncthreads();
        for (int64_t t = u.T - 1; t >= 0; --t) {
            const double omega = om_[t];
            const double tau = eta / omega, sigma = eta * omega;
            if (t < u.T - 1) {
                if (rs_[t]) {
                    for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                        bxh[j] = bx[j] + bx0[j];
                        bx[j] = 0.0;
                        bx0[j] = 0.0;
                    }
                    for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                        byh[i] = by[i] + by0[i];
                        by[i] = 0.0;
                        by0[i] = 0.0;
                    }
                } else {
                    const int64_t k = kk_[t];
                    const double ak = (double)(k + 1) / (double)(k + 2), bk = 1.0 / (double)(k + 2);
                    for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                        const double v = bx[j];
                        bxh[j] = ak * (1.0 + gam) * v;
                        bx0[j] += bk * v;
                        bx[j] = -ak * gam * v;
                    }
                    for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                        const double v = by[i];
                        byh[i] = ak * (1.0 + gam) * v;
                        by0[i] += bk * v;
                        by[i] = -ak * gam * v;
                    }
                }
            }
            // dual step: yhat = sigma (v - clamp(v, -u_c, -l_c)), v = y/sigma - A~ xext
            const uint64_t *ymt = ym + (size_t)t * 2 * yw;
            for (int32_t i = threadIdx.x; i < g.m; i += BT) {
                const uint64_t bit = 1ull << (i & 63);
                const bool at_u = (ymt[2 * (i >> 6)] & bit) != 0;
                const bool at_l = (ymt[2 * (i >> 6) + 1] & bit) != 0;
                const double bv = (at_u || at_l) ? sigma * byh[i] : 0.0;
                if (at_u) guc[i] += sigma * byh[i];
                if (at_l) glc[i] += sigma * byh[i];
                by[i] += bv / sigma;
                ba[i] = -bv;
            }
            __syncthreads();
            // xext = 2 xhat - x, then the primal step xhat = clamp(x - tau (c - A~'y))
            const uint64_t *xmt = xm + (size_t)t * xw;
            for (int32_t j = threadIdx.x; j < g.n; j += BT) {
                const double bxe = ONCHIP ? sell_dot(a.tsp, a.tsci, a.tsva, ts0 + (j >> 6), j & 63, ba)
                                          : csr_dot(trp, tci, tva, j, ba);
                const double bh = bxh[j] + 2.0 * bxe;
                bx[j] -= bxe;
                const bool inside = (xmt[j >> 6] >> (j & 63)) & 1ull;
                const double bu = inside ? bh : 0.0;
                bx[j] += bu;
                gc[j] += -tau * bu;
                tmp[j] = tau * bu;
            }
            __syncthreads();
            for (int32_t i = threadIdx.x; i < g.m; i += BT)
                by[i] += ONCHIP ? sell_dot(a.asp, a.asci, a.asva, as0 + (i >> 6), i & 63, tmp)
                                : csr_dot(arp, aci, ava, i, tmp);
            __syncthreads();
        }
        // c~ = D_c c, l~_c = D_r l_c, u~_c = D_r u_c
        for (int32_t j = threadIdx.x; j < g.n; j += BT) gc[j] = Dc[j] * gc[j];
        for (int32_t i = threadIdx.x; i < g.m; i += BT) {
            glc[i] = isfinite(a.lc_o[g.vr + i]) ? Dr[i] * glc[i] : 0.0;
            guc[i] = isfinite(a.uc_o[g.vr + i]) ? Dr[i] * guc[i] : 0.0;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// layout kernels

// Instance-local column indices of A and the row -> instance map check.
__global__ __launch_bounds__(kBlock) void k_batch_localize(const int32_t *__restrict__ row_off,
                                                           const int32_t *__restrict__ col_off,
                                                           int32_t B, const int32_t *__restrict__ rowptr,
                                                           int32_t *__restrict__ colidx,
                                                           int32_t *__restrict__ flag) {
    // one workgroup per instance, its rows strided over the threads
    const int32_t b = blockIdx.x;
    if (b >= B) return;
    const int32_t c0 = col_off[b], c1 = col_off[b + 1];
    if (row_off[b + 1] < row_off[b] || c1 <= c0) {
        if (threadIdx.x == 0) atomicOr(flag, 32);
        return;
    }
    for (int32_t i = row_off[b] + (int32_t)threadIdx.x; i < row_off[b + 1]; i += kBlock)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int32_t j = colidx[e];
            if (j < c0 || j >= c1) atomicOr(flag, 64);
            colidx[e] = j - c0;
        }
}

// Column indices of A' (global rows) made instance-local.
__global__ __launch_bounds__(kBlock) void k_batch_localize_t(const int32_t *__restrict__ row_off,
                                                             const int32_t *__restrict__ col_off,
                                                             int32_t B, const int32_t *__restrict__ trp,
                                                             int32_t *__restrict__ tci) {
    const int32_t b = blockIdx.x;
    if (b >= B) return;
    const int32_t r0 = row_off[b];
    for (int32_t j = col_off[b] + (int32_t)threadIdx.x; j < col_off[b + 1]; j += kBlock)
        for (int32_t e = trp[j]; e < trp[j + 1]; ++e) tci[e] -= r0;
}

}  // namespace pdhg

// ---------------------------------------------------------------------------
// host side

namespace pdhg {

static BOpts batch_opts(const pdhg_options &o) {
    BOpts b;
    b.eps = o.eps;
    b.gamma = o.gamma;
    b.step_safety = o.step_safety;
    b.beta_suff = o.restart_sufficient;
    b.beta_nec = o.restart_necessary;
    b.beta_art = o.restart_artificial;
    b.power_tol = o.power_tol;
    b.limit = std::min<int64_t>(o.iteration_limit, 10000000);
    b.check_every = o.check_every;
    b.ruiz_iters = o.ruiz_iters;
    b.pock_chambolle = o.pock_chambolle;
    b.power_max_iters = o.power_max_iters;
    b.eps_pinf = o.eps_primal_infeasible;
    b.eps_dinf = o.eps_dual_infeasible;
    b.detect = o.eps_primal_infeasible > 0.0 || o.eps_dual_infeasible > 0.0;
    b.pad = 0;
    return b;
}

static BArgs batch_args(BatchHandle &h) {
    BArgs a;
    memset(&a, 0, sizeof(a));
    a.B = h.B;
    a.shared = h.shared;
    a.m = h.m;
    a.n = h.n;
    a.row_off = h.row_off.p;
    a.col_off = h.col_off.p;
    a.arp = h.arp.p;
    a.aci = h.aci.p;
    a.ava = h.ava.p;
    a.trp = h.trp.p;
    a.tci = h.tci.p;
    a.tva = h.tva.p;
    a.Dr = h.Dr.p;
    a.Dc = h.Dc.p;
    a.eta = h.eta.p;
    a.power_iters = h.power_iters.p;
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
    a.x = h.x.p;
    a.x0 = h.x0.p;
    a.xh = h.xh.p;
    a.xe = h.xe.p;
    a.aty = h.aty.p;
    a.y = h.y.p;
    a.y0 = h.y0.p;
    a.yh = h.yh.p;
    a.res = h.res.p;
    a.queue = h.queue.p;
    a.x_init = h.x_init_;
    a.y_init = h.y_init_;
    a.asp = h.asp.p;
    a.asci = h.asci.p;
    a.asva = h.asva.p;
    a.asfirst = h.asfirst.p;
    a.tsp = h.tsp.p;
    a.tsci = h.tsci.p;
    a.tsva = h.tsva.p;
    a.tsfirst = h.tsfirst.p;
    a.lhist = h.lhist.p;
    a.p0 = h.rp0.p;
    a.q0 = h.rq0.p;
    a.ph = h.rph.p;
    a.qh = h.rqh.p;
    a.x_out = h.x_out_;
    a.y_out = h.y_out_;
    return a;
}

template <int BT>
static int32_t resident(const void *kernel) {
    int dev = 0, per_cu = 0;
    PDHG_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    PDHG_HIP(hipGetDeviceProperties(&prop, dev));
    PDHG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, BT, 0));
    return std::max(1, per_cu) * prop.multiProcessorCount;
}



// Dynamic LDS one workgroup may take (160 KB on gfx950), read once.
static size_t lds_per_workgroup() {
    static const size_t v = [] {
        int dev = 0, bytes = 0;
        PDHG_HIP(hipGetDevice(&dev));
        PDHG_HIP(hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        return (size_t)bytes;
    }();
    return v;
}

// Columns per thread of the register-resident kernels at BT threads (4 with
// one row slice, 8 with two), or 0 when the batch does not qualify: a shared
// matrix with narrow slices, BT >= 256, and x_ext, y, the row data and the
// column anchor, cost and upper bound in one workgroup's LDS.
template <int BT>
static int res_columns(const BatchHandle &h) {
    if (!(h.onchip && h.resident && h.shared && h.ts_wmax >= 1 && h.ts_wmax <= kResCol &&
          h.as_wmax <= kResRow && BT >= 256))
        return 0;
    if ((4 * (size_t)h.nmax + 4 * (size_t)h.mmax) * sizeof(double) > lds_per_workgroup()) return 0;
    if (h.nmax <= 4 * BT && h.mmax <= BT) return 4;
    if (h.nmax <= 8 * BT && h.mmax <= 2 * BT) return 8;
    return 0;
}

template <int BT, int S, bool RES>
static void launch_solve_lds_t(BatchHandle &h, const BOpts &o, BArgs a, size_t lds) {
    const void *kern = o.detect ? reinterpret_cast<const void *>(&k_batch_solve_lds<BT, S, RES, true>)
                                : reinterpret_cast<const void *>(&k_batch_solve_lds<BT, S, RES, false>);
    int dev = 0, per_cu = 0;
    PDHG_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    PDHG_HIP(hipGetDeviceProperties(&prop, dev));
    PDHG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BT, lds));
    int32_t wg = std::min(h.B, std::max(1, per_cu) * prop.multiProcessorCount);
    if (h.workgroups > 0) wg = std::min(wg, h.workgroups);
    PDHG_HIP(hipMemsetAsync(h.queue.p, 0, sizeof(int32_t), h.stream));
    if (o.detect)
        k_batch_solve_lds<BT, S, RES, true><<<wg, BT, lds, h.stream>>>(a, o, h.nmax, h.mmax);
    else
        k_batch_solve_lds<BT, S, RES, false><<<wg, BT, lds, h.stream>>>(a, o, h.nmax, h.mmax);
    PDHG_HIP(hipGetLastError());
}

template <class T>
static void load(DBuf<T> &dst, const T *src, size_t count, int mem, hipStream_t s);

// SELL-64 copy of a batch matrix (rows of every instance padded to whole
// slices) from the scaled CSR after the setup kernel: slice widths on the
// device, their prefix sum on the host (a few thousand slices), entries placed
// by one thread per slice row.
__global__ __launch_bounds__(kBlock) void k_sell_widths(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ r0,
                                                        const int32_t *__restrict__ r1, int32_t ns,
                                                        int32_t *__restrict__ width) {
    const int32_t sl = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (sl >= ns) return;
    int32_t w = 0;
    for (int32_t r = r0[sl]; r < r1[sl]; ++r) w = max(w, rp[r + 1] - rp[r]);
    width[sl] = w;
}

__global__ __launch_bounds__(kBlock) void k_sell_fill(const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const double *__restrict__ va,
                                                      const int32_t *__restrict__ r0,
                                                      const int32_t *__restrict__ r1,
                                                      const int32_t *__restrict__ sp, int32_t ns,
                                                      int32_t *__restrict__ sci,
                                                      double *__restrict__ sva) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int32_t sl = (int32_t)(t >> 6), lane = (int32_t)(t & 63);
    if (sl >= ns) return;
    const int32_t row = r0[sl] + lane;
    if (row >= r1[sl]) return;
    const int32_t e0 = rp[row], e1 = rp[row + 1];
    for (int32_t e = e0; e < e1; ++e) {
        const int64_t o = (int64_t)sp[sl] + 64 * (int64_t)(e - e0) + lane;
        sci[o] = ci[e];
        sva[o] = va[e];
    }
}

static int32_t build_batch_sell(hipStream_t s, int32_t nb, const std::vector<int32_t> &roff,
                                const DBuf<int32_t> &rp, const DBuf<int32_t> &ci, const DBuf<double> &va,
                                int64_t nnz, DBuf<int32_t> &sp, DBuf<int32_t> &sci, DBuf<double> &sva,
                                DBuf<int32_t> &sfirst) {
    (void)nnz;
    std::vector<int32_t> first((size_t)nb + 1), h0, h1;
    for (int32_t b = 0; b < nb; ++b) {
        first[b] = (int32_t)h0.size();
        for (int32_t r = roff[b]; r < roff[b + 1]; r += 64) {
            h0.push_back(r);
            h1.push_back(std::min(r + 64, roff[b + 1]));
        }
    }
    const int32_t ns = (int32_t)h0.size();
    first[nb] = ns;
    DBuf<int32_t> d0, d1, width;
    load(d0, h0.data(), h0.size(), PDHG_MEM_HOST, s);
    load(d1, h1.data(), h1.size(), PDHG_MEM_HOST, s);
    width.alloc((size_t)std::max(1, ns));
    std::vector<int32_t> hw((size_t)ns), off((size_t)ns + 1, 0);
    if (ns > 0) {
        k_sell_widths<<<(unsigned)ceil_div(ns, kBlock), kBlock, 0, s>>>(rp.p, d0.p, d1.p, ns, width.p);
        PDHG_HIP(hipMemcpyAsync(hw.data(), width.p, (size_t)ns * 4, hipMemcpyDeviceToHost, s));
        PDHG_HIP(hipStreamSynchronize(s));
    }
    int64_t total = 0;
    int32_t wmax = 0;
    for (int32_t i = 0; i < ns; ++i) {
        wmax = std::max(wmax, hw[i]);
        total += 64 * (int64_t)hw[i];
        if (total >= INT32_MAX) fail(PDHG_ERR_UNSUPPORTED, "batch matrix too large for 32-bit offsets");
        off[(size_t)i + 1] = (int32_t)total;
    }
    load(sp, off.data(), off.size(), PDHG_MEM_HOST, s);
    load(sfirst, first.data(), first.size(), PDHG_MEM_HOST, s);
    // at least one slice's worth: empty slices read the first 64 entries
    const size_t cap = (size_t)std::max<int64_t>(total, 64);
    sci.alloc(cap);
    sva.alloc(cap);
    PDHG_HIP(hipMemsetAsync(sci.p, 0, cap * 4, s));
    PDHG_HIP(hipMemsetAsync(sva.p, 0, cap * 8, s));
    if (ns > 0)
        k_sell_fill<<<(unsigned)ceil_div((int64_t)ns * 64, kBlock), kBlock, 0, s>>>(
            rp.p, ci.p, va.p, d0.p, d1.p, sp.p, ns, sci.p, sva.p);
    PDHG_HIP(hipGetLastError());
    PDHG_HIP(hipStreamSynchronize(s));
    return wmax;
}

// Largest instance column / row counts (LDS sizing of the on-chip solve).
static void instance_extents(BatchHandle &h) {
    if (h.shared) {
        h.nmax = h.n;
        h.mmax = h.m;
        return;
    }
    h.nmax = h.mmax = 0;
    for (int32_t b = 0; b < h.B; ++b) {
        h.nmax = std::max(h.nmax, h.col_off_h[b + 1] - h.col_off_h[b]);
        h.mmax = std::max(h.mmax, h.row_off_h[b + 1] - h.row_off_h[b]);
    }
}

// Default threads per instance: 1024 when the batch has at most one instance
// per compute unit, else the fewest (from 256) that keep the largest instance
// on chip with at most 8 columns and 8 rows per thread.
static int32_t default_threads(const BatchHandle &h) {
    int dev = 0, cus = 0;
    PDHG_HIP(hipGetDevice(&dev));
    PDHG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (h.B <= cus) return 1024;
    const int32_t need = std::max(h.nmax, h.mmax);
    int32_t bt = 256;
    while (bt < 1024 && 8 * bt < need) bt *= 2;
    return bt;
}

template <int BT>
static void launch_solve_t(BatchHandle &h, const BOpts &o) {
    BArgs a = batch_args(h);
    // on-chip variant when x_ext, y and the three per-row vectors fit the
    // workgroup's LDS and every thread owns at most 8 columns and 8 rows;
    // register-resident matrix for narrow shared slices when the rows fit
    // S/4 per thread (S >= 4) and the LDS also holds the column anchor, cost
    // and upper bound
    const size_t lds = ((size_t)h.nmax + 4 * (size_t)h.mmax) * sizeof(double);
    const size_t lds_res = lds + 3 * (size_t)h.nmax * sizeof(double);
    const int32_t need = std::max(h.nmax, h.mmax);
    if (h.onchip && lds <= lds_per_workgroup() && need <= 8 * BT) {
        const size_t l = std::max<size_t>(lds, 8);
        if (need <= BT) return launch_solve_lds_t<BT, 1, false>(h, o, a, l);
        if (need <= 2 * BT) return launch_solve_lds_t<BT, 2, false>(h, o, a, l);
        const bool res = h.resident && h.shared && h.ts_wmax <= kResCol && h.as_wmax <= kResRow &&
                         lds_res <= lds_per_workgroup() && BT >= 256;
        if (need <= 4 * BT) {
            if (res && h.mmax <= BT) return launch_solve_lds_t<BT, 4, true>(h, o, a, lds_res);
            return launch_solve_lds_t<BT, 4, false>(h, o, a, l);
        }
        if (res && h.mmax <= 2 * BT) return launch_solve_lds_t<BT, 8, true>(h, o, a, lds_res);
        return launch_solve_lds_t<BT, 8, false>(h, o, a, l);
    }

    int32_t wg = std::min(h.B, resident<BT>(o.detect ? reinterpret_cast<const void *>(&k_batch_solve<BT, true>)
                                                     : reinterpret_cast<const void *>(&k_batch_solve<BT, false>)));
    if (h.workgroups > 0) wg = std::min(wg, h.workgroups);
    PDHG_HIP(hipMemsetAsync(h.queue.p, 0, sizeof(int32_t), h.stream));
    if (o.detect)
        k_batch_solve<BT, true><<<wg, BT, 0, h.stream>>>(a, o);
    else
        k_batch_solve<BT, false><<<wg, BT, 0, h.stream>>>(a, o);
    PDHG_HIP(hipGetLastError());
}

// Dynamic LDS of the on-chip setup / unrolled / reverse kernels, or 0 when the
// largest instance does not fit (then the memory-resident variant runs).
static size_t onchip_lds(const BatchHandle &h) {
    const size_t lds = ((size_t)h.nmax + (size_t)h.mmax) * sizeof(double);
    return (h.onchip && lds <= 65536) ? std::max<size_t>(lds, 8) : 0;
}

template <int BT, class K>
static int32_t resident_lds(BatchHandle &h, K kernel, size_t lds) {
    int dev = 0, per_cu = 0;
    PDHG_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    PDHG_HIP(hipGetDeviceProperties(&prop, dev));
    PDHG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kernel), BT, lds));
    int32_t wg = std::min(h.B, std::max(1, per_cu) * prop.multiProcessorCount);
    if (h.workgroups > 0) wg = std::min(wg, h.workgroups);
    return wg;
}

template <int BT>
static void launch_setup_t(BatchHandle &h, int32_t count) {
    BArgs a = batch_args(h);
    const BOpts o = batch_opts(h.opt);
    const size_t lds = onchip_lds(h);
    PDHG_HIP(hipMemsetAsync(h.queue.p, 0, sizeof(int32_t), h.stream));
    if (lds) {
        const int32_t wg = std::min(count, resident_lds<BT>(h, &k_batch_setup<BT, true>, lds));
        k_batch_setup<BT, true><<<wg, BT, lds, h.stream>>>(a, o, count, h.nmax);
    } else {
        const int32_t wg = std::min(count, resident_lds<BT>(h, &k_batch_setup<BT, false>, 0));
        k_batch_setup<BT, false><<<wg, BT, 0, h.stream>>>(a, o, count, 0);
    }
    PDHG_HIP(hipGetLastError());
}

// The setup (scaling sweeps and power iteration, one workgroup per instance)
// is latency-bound: it runs with about two columns per thread whatever the
// solve's launch shape, between 256 and 1024 threads.
static void dispatch_setup(BatchHandle &h, int32_t count) {
    const int32_t need = std::max(h.nmax, h.mmax);
    int32_t bt = 256;
    while (bt < 1024 && 2 * bt < need) bt *= 2;
    switch (bt) {
        case 64: launch_setup_t<64>(h, count); break;
        case 128: launch_setup_t<128>(h, count); break;
        case 512: launch_setup_t<512>(h, count); break;
        case 1024: launch_setup_t<1024>(h, count); break;
        default: launch_setup_t<256>(h, count); break;
    }
}

// Solves that test infeasibility rays carry a larger register budget: the
// 1024-thread variants spill, so the default launch takes at most 512 there.
static void dispatch_solve(BatchHandle &h, const BOpts &o) {
    const int32_t threads = (o.detect && !h.threads_set) ? std::min(h.threads, 512) : h.threads;
    switch (threads) {
        case 64: launch_solve_t<64>(h, o); break;
        case 128: launch_solve_t<128>(h, o); break;
        case 512: launch_solve_t<512>(h, o); break;
        case 1024: launch_solve_t<1024>(h, o); break;
        default: launch_solve_t<256>(h, o); break;
    }
}

template <class T>
static void load(DBuf<T> &dst, const T *src, size_t count, int mem, hipStream_t s) {
    dst.alloc(count);
    if (count == 0) return;
    PDHG_HIP(hipMemcpyAsync(dst.p, src, count * sizeof(T),
                            mem == PDHG_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                   : hipMemcpyHostToDevice,
                            s));
}

BatchHandle *batch_create(const pdhg_batch_problem &p, const pdhg_options &o, void *stream) {
    if (p.batch < 1 || (p.shared_a != 0 && p.shared_a != 1) || p.m < 0 || p.n < 1)
        fail(PDHG_ERR_INVALID_ARG, "need batch >= 1, shared_a in {0,1}, m >= 0, n >= 1");
    if (p.mem != PDHG_MEM_HOST && p.mem != PDHG_MEM_DEVICE)
        fail(PDHG_ERR_INVALID_ARG, "mem must be PDHG_MEM_HOST or PDHG_MEM_DEVICE");
    if (!p.a_rowptr || (p.a_nnz > 0 && (!p.a_colidx || !p.a_val)) || p.a_nnz < 0 ||
        p.a_nnz >= INT32_MAX)
        fail(PDHG_ERR_INVALID_ARG, "bad CSR arrays or nnz");
    if (!p.c || !p.lv || !p.uv || (p.m > 0 && (!p.lc || !p.uc)))
        fail(PDHG_ERR_INVALID_ARG, "NULL objective or bound vector");
    if (!p.shared_a && (!p.row_off || !p.col_off))
        fail(PDHG_ERR_INVALID_ARG, "ragged batches need row_off and col_off");
    if (p.shared_a && ((int64_t)p.batch * p.n >= INT32_MAX || (int64_t)p.batch * p.m >= INT32_MAX))
        fail(PDHG_ERR_UNSUPPORTED, "batch vectors exceed 32-bit indexing");
    auto hp = std::make_unique<BatchHandle>();
    BatchHandle &h = *hp;
    const double t0 = now_seconds();
    h.B = p.batch;
    h.shared = p.shared_a;
    h.m = p.m;
    h.n = p.n;
    h.nnz = p.a_nnz;
    h.opt = o;
    h.vec_m = h.shared ? h.B * h.m : h.m;
    h.vec_n = h.shared ? h.B * h.n : h.n;
    PDHG_HIP(hipStreamCreateWithFlags(&h.stream, hipStreamNonBlocking));
    PDHG_HIP(hipEventCreateWithFlags(&h.ev, hipEventDisableTiming));
    order_after_stream(h.stream, h.ev, stream);
    hipStream_t s = h.stream;

    load(h.arp, p.a_rowptr, (size_t)h.m + 1, p.mem, s);
    load(h.aci, p.a_colidx, (size_t)h.nnz, p.mem, s);
    load(h.ava, p.a_val, (size_t)h.nnz, p.mem, s);
    validate_csr(s, h.arp.p, h.aci.p, h.ava.p, h.m, h.n, h.nnz);
    if (!h.shared) {
        std::vector<int32_t> ro((size_t)h.B + 1), co((size_t)h.B + 1);
        if (p.mem == PDHG_MEM_DEVICE) {
            PDHG_HIP(hipMemcpy(ro.data(), p.row_off, ro.size() * 4, hipMemcpyDeviceToHost));
            PDHG_HIP(hipMemcpy(co.data(), p.col_off, co.size() * 4, hipMemcpyDeviceToHost));
        } else {
            memcpy(ro.data(), p.row_off, ro.size() * 4);
            memcpy(co.data(), p.col_off, co.size() * 4);
        }
        if (ro[0] != 0 || co[0] != 0 || ro[h.B] != h.m || co[h.B] != h.n)
            fail(PDHG_ERR_INVALID_INPUT, "row_off / col_off must start at 0 and end at m / n");
        for (int32_t b = 0; b < h.B; ++b)
            if (ro[b + 1] < ro[b] || co[b + 1] <= co[b])
                fail(PDHG_ERR_INVALID_INPUT, "instance offsets must increase (>= 1 column each)");
        load(h.row_off, ro.data(), ro.size(), PDHG_MEM_HOST, s);
        load(h.col_off, co.data(), co.size(), PDHG_MEM_HOST, s);
        h.row_off_h = ro;
        h.col_off_h = co;
    } else {
        h.row_off.alloc(1);
        h.col_off.alloc(1);
    }
    instance_extents(h);
    h.threads = default_threads(h);
    // A' from the global matrix, then instance-local indices on both
    h.trp.alloc((size_t)h.n + 1);
    h.tci.alloc((size_t)h.nnz);
    h.tva.alloc((size_t)h.nnz);
    plain_transpose(s, h.m, h.n, h.nnz, h.arp.p, h.aci.p, h.ava.p, h.trp.p, h.tci.p, h.tva.p);
    if (!h.shared) {
        DBuf<int32_t> flag;
        flag.alloc(1);
        PDHG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
        const unsigned nb = (unsigned)h.B;
        k_batch_localize<<<nb, kBlock, 0, s>>>(h.row_off.p, h.col_off.p, h.B, h.arp.p, h.aci.p,
                                                flag.p);
        check_flag(s, flag.p, "a ragged instance has entries outside its column range");
        k_batch_localize_t<<<nb, kBlock, 0, s>>>(h.row_off.p, h.col_off.p, h.B, h.trp.p, h.tci.p);
    }
    load(h.c_o, p.c, (size_t)h.vec_n, p.mem, s);
    load(h.lv_o, p.lv, (size_t)h.vec_n, p.mem, s);
    load(h.uv_o, p.uv, (size_t)h.vec_n, p.mem, s);
    load(h.lc_o, p.lc, (size_t)h.vec_m, p.mem, s);
    load(h.uc_o, p.uc, (size_t)h.vec_m, p.mem, s);
    validate_vectors(s, h.vec_n, h.vec_m, h.c_o.p, h.lv_o.p, h.uv_o.p, h.lc_o.p, h.uc_o.p);
    for (auto *b : {&h.c, &h.lv, &h.uv, &h.x, &h.x0, &h.xh, &h.xe, &h.aty}) b->alloc((size_t)h.vec_n);
    for (auto *b : {&h.lc, &h.uc, &h.y, &h.y0, &h.yh}) b->alloc((size_t)h.vec_m);
    h.Dr.alloc((size_t)h.m);
    h.Dc.alloc((size_t)h.n);
    const int32_t nscal = h.shared ? 1 : h.B;
    h.eta.alloc((size_t)nscal);
    h.power_iters.alloc((size_t)nscal);
    h.res.alloc((size_t)h.B);
    h.queue.alloc(1);
    h.lhist.alloc((size_t)nscal * 2 * ((size_t)std::max(1, o.power_max_iters) + 1));
    if (p.q_rank == 0) {   // LP batches test infeasibility rays at checks
        for (auto *b : {&h.rq0, &h.rqh}) b->alloc((size_t)h.vec_n);
        for (auto *b : {&h.rp0, &h.rph}) b->alloc((size_t)std::max(1, h.vec_m));
    }
    dispatch_setup(h, nscal);
    PDHG_HIP(hipStreamSynchronize(s));
    h.lhist.release();
    {
        const int32_t nb = h.shared ? 1 : h.B;
        std::vector<int32_t> ro = h.shared ? std::vector<int32_t>{0, h.m} : h.row_off_h;
        std::vector<int32_t> co = h.shared ? std::vector<int32_t>{0, h.n} : h.col_off_h;
        h.as_wmax = build_batch_sell(s, nb, ro, h.arp, h.aci, h.ava, h.nnz, h.asp, h.asci, h.asva, h.asfirst);
        h.ts_wmax = build_batch_sell(s, nb, co, h.trp, h.tci, h.tva, h.nnz, h.tsp, h.tsci, h.tsva, h.tsfirst);
    }
    // one instance per CU would take 1024 threads; a matrix that the
    // register-resident kernels can hold runs faster at 512 (their 1024-thread
    // variants spill)
    if (p.q_rank == 0 && h.threads == 1024 && res_columns<512>(h)) h.threads = 512;
    if (p.q_rank > 0) bqp_create(h, p);
    h.setup_seconds = now_seconds() - t0;
    return hp.release();
}

void batch_solve(BatchHandle &h, const double *x_init, const double *y_init, double *x_out,
                 double *y_out, pdhg_result *res) {
    if (h.q_rank > 0) {
        bqp_solve(h, x_init, y_init, x_out, y_out, res);
        return;
    }
    const double t0 = now_seconds();
    BOpts o = batch_opts(h.opt);
    // pointers of this call go in through the argument block
    h.x_init_ = x_init;
    h.y_init_ = y_init;
    h.x_out_ = x_out;
    h.y_out_ = y_out;
    dispatch_solve(h, o);
    PDHG_HIP(hipStreamSynchronize(h.stream));
    const double el = now_seconds() - t0;
    if (res) {
        std::vector<BatchRes> r((size_t)h.B);
        PDHG_HIP(hipMemcpy(r.data(), h.res.p, sizeof(BatchRes) * h.B, hipMemcpyDeviceToHost));
        for (int32_t b = 0; b < h.B; ++b) {
            pdhg_result &q = res[b];
            memset(&q, 0, sizeof(q));
            q.status = r[b].status;
            q.iterations = r[b].iterations;
            q.restarts = r[b].restarts;
            q.primal_obj = r[b].pobj;
            q.dual_obj = r[b].dobj;
            q.rel_primal_res = r[b].rel_p;
            q.rel_dual_res = r[b].rel_d;
            q.rel_gap = r[b].rel_g;
            q.kkt_rel = r[b].kkt;
            q.solve_seconds = el;
            q.setup_seconds = h.setup_seconds;
            q.eta = r[b].eta;
            q.omega = r[b].omega;
            q.norm_a = r[b].eta > 0.0 ? h.opt.step_safety / r[b].eta : 0.0;
            q.power_iters = r[b].power_iters;
        }
    }
}

void batch_set_launch(BatchHandle &h, int32_t threads, int32_t workgroups) {
    if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
        fail(PDHG_ERR_INVALID_ARG, "threads must be 64, 128, 256, 512 or 1024");
    h.threads = threads;
    h.threads_set = true;
    h.workgroups = workgroups;
}

int32_t batch_autotune(BatchHandle &h, int32_t iterations) {
    // Every trial runs with the limit `iterations` into temporary outputs; the
    // caller's limit, launch shape and output pointers come back even if a
    // trial fails, and the best thread count is kept only on success.
    struct Restore {
        BatchHandle &h;
        int64_t limit;
        int32_t threads;
        bool set;
        const double *x_init, *y_init;
        double *x_out, *y_out;
        ~Restore() {
            h.opt.iteration_limit = limit;
            h.threads = threads;
            h.threads_set = set;
            h.x_init_ = x_init;
            h.y_init_ = y_init;
            h.x_out_ = x_out;
            h.y_out_ = y_out;
        }
    } restore{h, h.opt.iteration_limit, h.threads, h.threads_set,
              h.x_init_, h.y_init_, h.x_out_, h.y_out_};
    DBuf<double> xo, yo;
    xo.alloc((size_t)h.vec_n);
    yo.alloc((size_t)std::max(1, h.vec_m));
    const bool qp = h.q_rank > 0;
    BOpts o = batch_opts(h.opt);
    o.limit = iterations;
    h.opt.iteration_limit = iterations;
    h.x_out_ = xo.p;
    h.y_out_ = yo.p;
    h.x_init_ = nullptr;
    h.y_init_ = nullptr;
    auto trial = [&]() {
        if (qp) bqp_solve(h, nullptr, nullptr, xo.p, yo.p, nullptr);
        else dispatch_solve(h, o);
        PDHG_HIP(hipStreamSynchronize(h.stream));
    };
    int32_t best = h.threads;
    double best_t = 1e300;
    h.threads_set = true;   // each trial runs the thread count it names
    for (int32_t t : {64, 128, 256, 512, 1024}) {
        h.threads = t;
        trial();   // warm-up
        const double t0 = now_seconds();
        trial();
        const double el = now_seconds() - t0;
        if (el < best_t) {
            best_t = el;
            best = t;
        }
    }
    restore.threads = best;
    restore.set = true;
    return best;
}

static UArgs unrolled_args(BatchHandle &h) {
    UArgs u;
    memset(&u, 0, sizeof(u));
    u.T = h.unrolled_T;
    u.restart = h.u_restart.p;
    u.omega = h.u_omega.p;
    u.kk = h.u_kk.p;
    u.xmask = h.u_xmask.p;
    u.ymask = h.u_ymask.p;
    u.xm_off = h.u_xoff.p;
    u.ym_off = h.u_yoff.p;
    u.ba = h.u_ba.p;
    return u;
}

template <int BT>
static void launch_unrolled_t(BatchHandle &h, const UArgs &u) {
    BArgs a = batch_args(h);
    const BOpts o = batch_opts(h.opt);
    const size_t lds = onchip_lds(h);
    PDHG_HIP(hipMemsetAsync(h.queue.p, 0, sizeof(int32_t), h.stream));
    if constexpr (BT == 256 || BT == 512) {
        const int rc = res_columns<BT>(h);
        if (rc) {
            const size_t l = (4 * (size_t)h.nmax + 4 * (size_t)h.mmax) * sizeof(double);
            if (rc == 4) {
                const int32_t wg = resident_lds<BT>(h, &k_batch_unrolled_res<BT, 4>, l);
                k_batch_unrolled_res<BT, 4><<<wg, BT, l, h.stream>>>(a, o, u, h.nmax, h.mmax);
            } else {
                const int32_t wg = resident_lds<BT>(h, &k_batch_unrolled_res<BT, 8>, l);
                k_batch_unrolled_res<BT, 8><<<wg, BT, l, h.stream>>>(a, o, u, h.nmax, h.mmax);
            }
            PDHG_HIP(hipGetLastError());
            return;
        }
    }
    if (lds) {
        const int32_t wg = resident_lds<BT>(h, &k_batch_unrolled<BT, true>, lds);
        k_batch_unrolled<BT, true><<<wg, BT, lds, h.stream>>>(a, o, u, h.nmax);
    } else {
        const int32_t wg = resident_lds<BT>(h, &k_batch_unrolled<BT, false>, 0);
        k_batch_unrolled<BT, false><<<wg, BT, 0, h.stream>>>(a, o, u, 0);
    }
    PDHG_HIP(hipGetLastError());
}

template <int BT>
static void launch_backward_t(BatchHandle &h, const UArgs &u) {
    BArgs a = batch_args(h);
    const BOpts o = batch_opts(h.opt);
    const size_t lds = onchip_lds(h);
    PDHG_HIP(hipMemsetAsync(h.queue.p, 0, sizeof(int32_t), h.stream));
    if constexpr (BT == 256 || BT == 512) {
        const int rc = res_columns<BT>(h);
        if (rc) {
            const size_t l = ((size_t)h.nmax + (size_t)h.mmax) * sizeof(double);
            if (rc == 4) {
                const int32_t wg = resident_lds<BT>(h, &k_batch_backward_res<BT, 4>, l);
                k_batch_backward_res<BT, 4><<<wg, BT, l, h.stream>>>(a, o, u, h.nmax);
            } else {
                const int32_t wg = resident_lds<BT>(h, &k_batch_backward_res<BT, 8>, l);
                k_batch_backward_res<BT, 8><<<wg, BT, l, h.stream>>>(a, o, u, h.nmax);
            }
            PDHG_HIP(hipGetLastError());
            return;
        }
    }
    if (lds) {
        const int32_t wg = resident_lds<BT>(h, &k_batch_backward<BT, true>, lds);
        k_batch_backward<BT, true><<<wg, BT, lds, h.stream>>>(a, o, u, h.nmax);
    } else {
        const int32_t wg = resident_lds<BT>(h, &k_batch_backward<BT, false>, 0);
        k_batch_backward<BT, false><<<wg, BT, 0, h.stream>>>(a, o, u, 0);
    }
    PDHG_HIP(hipGetLastError());
}

void batch_unrolled_forward(BatchHandle &h, int64_t T, int32_t replay, double *x_out,
                            double *y_out) {
    if (h.q_rank > 0) {
        bqp_unrolled(h, T, replay, x_out, y_out);
        return;
    }
    if (T < 1 || T > 1000000) fail(PDHG_ERR_INVALID_ARG, "T must be in [1, 10^6]");
    if (replay && h.unrolled_T != T)
        fail(PDHG_ERR_INVALID_ARG, "replay needs a recorded schedule of the same length T");
    if (h.unrolled_T != T) {
        // per-instance mask offsets (64-bit words)
        std::vector<int64_t> xo((size_t)h.B + 1, 0), yo((size_t)h.B + 1, 0);
        for (int32_t b = 0; b < h.B; ++b) {
            const int64_t n_b = h.shared ? h.n : h.col_off_h[b + 1] - h.col_off_h[b];
            const int64_t m_b = h.shared ? h.m : h.row_off_h[b + 1] - h.row_off_h[b];
            xo[b + 1] = xo[b] + ((n_b + 63) / 64) * T;
            yo[b + 1] = yo[b] + 2 * ((m_b + 63) / 64) * T;
        }
        h.u_xoff.alloc(xo.size());
        h.u_yoff.alloc(yo.size());
        PDHG_HIP(hipMemcpy(h.u_xoff.p, xo.data(), xo.size() * 8, hipMemcpyHostToDevice));
        PDHG_HIP(hipMemcpy(h.u_yoff.p, yo.data(), yo.size() * 8, hipMemcpyHostToDevice));
        h.u_xmask.alloc((size_t)std::max<int64_t>(1, xo[h.B]));
        h.u_ymask.alloc((size_t)std::max<int64_t>(1, yo[h.B]));
        h.u_restart.alloc((size_t)h.B * T);
        h.u_omega.alloc((size_t)h.B * T);
        h.u_kk.alloc((size_t)h.B * T);
        h.u_ba.alloc((size_t)std::max(1, h.vec_m));
        h.unrolled_T = T;
    }
    h.x_out_ = x_out;
    h.y_out_ = y_out;
    UArgs u = unrolled_args(h);
    u.replay = replay;
    switch (h.threads) {
        case 64: launch_unrolled_t<64>(h, u); break;
        case 128: launch_unrolled_t<128>(h, u); break;
        case 512: launch_unrolled_t<512>(h, u); break;
        case 1024: launch_unrolled_t<1024>(h, u); break;
        default: launch_unrolled_t<256>(h, u); break;
    }
    PDHG_HIP(hipStreamSynchronize(h.stream));
}

void batch_backward(BatchHandle &h, const double *gx, const double *gy, double *gc, double *glc,
                    double *guc, double *gd) {
    if (h.q_rank > 0) {
        bqp_backward(h, gx, gy, gc, glc, guc, gd);
        return;
    }
    if (h.unrolled_T < 1) fail(PDHG_ERR_INVALID_ARG, "run pdhg_batch_unrolled_forward first");
    DBuf<double> zm, lcs, ucs;
    zm.alloc((size_t)std::max(1, h.vec_m));
    PDHG_HIP(hipMemsetAsync(zm.p, 0, sizeof(double) * std::max(1, h.vec_m), h.stream));
    // gradients of rows without bounds are written to scratch when not requested
    lcs.alloc((size_t)std::max(1, h.vec_m));
    ucs.alloc((size_t)std::max(1, h.vec_m));
    UArgs u = unrolled_args(h);
    u.gx = gx;
    u.gy = gy ? gy : zm.p;
    u.gc = gc;
    u.glc = glc ? glc : lcs.p;
    u.guc = guc ? guc : ucs.p;
    switch (h.threads) {
        case 64: launch_backward_t<64>(h, u); break;
        case 128: launch_backward_t<128>(h, u); break;
        case 512: launch_backward_t<512>(h, u); break;
        case 1024: launch_backward_t<1024>(h, u); break;
        default: launch_backward_t<256>(h, u); break;
    }
    PDHG_HIP(hipStreamSynchronize(h.stream));
}

void batch_update_data(BatchHandle &h, const double *c, const double *lc, const double *uc,
                       const double *lv, const double *uv) {
    hipStream_t s = h.stream;
    DBuf<double> nc, nlc, nuc, nlv, nuv;
    auto take = [&](DBuf<double> &dst, const double *src, const DBuf<double> &cur, int32_t len) {
        dst.alloc((size_t)std::max(1, len));
        PDHG_HIP(hipMemcpyAsync(dst.p, src ? src : cur.p, sizeof(double) * (size_t)len,
                                hipMemcpyDeviceToDevice, s));
    };
    take(nc, c, h.c_o, h.vec_n);
    take(nlv, lv, h.lv_o, h.vec_n);
    take(nuv, uv, h.uv_o, h.vec_n);
    take(nlc, lc, h.lc_o, h.vec_m);
    take(nuc, uc, h.uc_o, h.vec_m);
    validate_vectors(s, h.vec_n, h.vec_m, nc.p, nlv.p, nuv.p, nlc.p, nuc.p);
    std::swap(h.c_o.p, nc.p);
    std::swap(h.lv_o.p, nlv.p);
    std::swap(h.uv_o.p, nuv.p);
    std::swap(h.lc_o.p, nlc.p);
    std::swap(h.uc_o.p, nuc.p);
    PDHG_HIP(hipStreamSynchronize(s));
}

void batch_destroy(BatchHandle *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

}  // namespace pdhg
