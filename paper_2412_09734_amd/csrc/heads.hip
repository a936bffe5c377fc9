// Loss heads around the unrolled solver for end-to-end learning (Section 4,
// the shortest-path and portfolio pipelines): a linear cost model on
// per-variable features, the regret of the decisions under the true costs,
// the weight gradient of the cost model, and the value / gradient of a
// low-rank-plus-diagonal QP objective. All sums are deterministic
// workgroup trees in a fixed order.
#include <algorithm>
#include <mutex>

#include "device.hpp"

namespace pdhg {

constexpr int kHeadChunks = 64;   // column chunks of the weight-gradient reduction
constexpr int kHeadRmax = 32;     // largest factor rank of pdhg_qp_value
constexpr int kHeadPmax = 64;     // most features of the linear cost model
constexpr int kScratchDoubles = kHeadPmax * kHeadChunks;
constexpr int kMaxDevices = 64;

// Partial sums of the allocation-free weight gradient (32 KB on every GPU the
// library runs on, kept until the process ends). Host code never uses this
// name as an address: it reads the device address once per device with
// hipGetSymbolAddress and passes that to the kernels.
static __device__ __align__(256) double scratch[kScratchDoubles];

__global__ __launch_bounds__(kBlock) void k_linear_costs(int64_t N, int32_t p,
                                                         const double *__restrict__ f,
                                                         const double *__restrict__ W,
                                                         double *__restrict__ c) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int32_t k = 0; k < p; ++k) s = fma(W[k], f[i * p + k], s);
    c[i] = s;
}

// One workgroup per instance: loss[b] = c_true_b' x_b - v_star[b].
__global__ __launch_bounds__(kBlock) void k_regret(int32_t n, const double *__restrict__ ct,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ vs,
                                                   double *__restrict__ loss) {
    const int32_t b = blockIdx.x;
    const size_t o = (size_t)b * n;
    double v[1] = {0.0};
    for (int32_t a = threadIdx.x; a < n; a += kBlock) v[0] = fma(ct[o + a], x[o + a], v[0]);
    block_sum_all<1>(v);
    if (threadIdx.x == 0) loss[b] = v[0] - vs[b];
}

// Partial weight gradients: workgroup (k, chunk) sums gc[i] f[i, k] over
// chunk `chunk` of the N = B n entries into part[k * kHeadChunks + chunk].
__global__ __launch_bounds__(kBlock) void k_costs_grad_part(int64_t N, int32_t p,
                                                            const double *__restrict__ f,
                                                            const double *__restrict__ gc,
                                                            double *__restrict__ part) {
    const int32_t k = blockIdx.x / kHeadChunks, chunk = blockIdx.x % kHeadChunks;
    const int64_t len = (N + kHeadChunks - 1) / kHeadChunks;
    const int64_t i0 = chunk * len, i1 = std::min(N, i0 + len);
    double v[1] = {0.0};
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) v[0] = fma(gc[i], f[i * p + k], v[0]);
    block_sum_store<1>(v, part + (size_t)k * kHeadChunks + chunk);
}

__global__ __launch_bounds__(64) void k_costs_grad_final(int32_t p, const double *__restrict__ part,
                                                         double *__restrict__ gW) {
    const int32_t k = threadIdx.x;
    if (k >= p) return;
    double s = 0.0;
    for (int32_t q = 0; q < kHeadChunks; ++q) s += part[(size_t)k * kHeadChunks + q];
    gW[k] = s;
}

// One workgroup per instance: t = F' x, Qx = F t + d x, value and gradient.
__global__ __launch_bounds__(kBlock) void k_qp_value(int32_t n, int32_t r, const double *__restrict__ F,
                                                     const double *__restrict__ d,
                                                     const double *__restrict__ c,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ value,
                                                     double *__restrict__ gx) {
    const int32_t b = blockIdx.x;
    const size_t o = (size_t)b * n;
    double t[kHeadRmax];
#pragma unroll
    for (int k = 0; k < kHeadRmax; ++k) t[k] = 0.0;
    for (int32_t j = threadIdx.x; j < n; j += kBlock) {
        const double xj = x[o + j];
        for (int32_t k = 0; k < r; ++k) t[k] = fma(F[(size_t)j * r + k], xj, t[k]);
    }
    block_sum_all<kHeadRmax>(t);
    double v[1] = {0.0};
    for (int32_t j = threadIdx.x; j < n; j += kBlock) {
        double qx = d[o + j] * x[o + j];
        for (int32_t k = 0; k < r; ++k) qx = fma(F[(size_t)j * r + k], t[k], qx);
        const double g = qx + c[o + j];
        if (gx) gx[o + j] = g;
        v[0] += x[o + j] * (0.5 * qx + c[o + j]);
    }
    block_sum_all<1>(v);
    if (threadIdx.x == 0) value[b] = v[0];
}

// SPO+ (Elmachtoub-Grigas) for min_{w in S} c'w: the inner problem's costs
// 2 c_hat - c_true, entrywise over the N = B n variables.
__global__ __launch_bounds__(kBlock) void k_spo_costs(int64_t N, const double *__restrict__ ch,
                                                      const double *__restrict__ ct,
                                                      double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < N) out[i] = 2.0 * ch[i] - ct[i];
}

// One workgroup per instance: with w* optimal under c_true (value z*) and w~
// optimal under 2 c_hat - c_true, loss = -(2 c_hat - c)'w~ + 2 c_hat'w* - z*,
// summed as 2 c_hat'(w* - w~) + c'w~ - z* (the same value, without the
// cancellation of two large products), and the subgradient 2 (w* - w~).
__global__ __launch_bounds__(kBlock) void k_spo_plus(int32_t n, const double *__restrict__ ch,
                                                     const double *__restrict__ ct,
                                                     const double *__restrict__ ws,
                                                     const double *__restrict__ zs,
                                                     const double *__restrict__ wt,
                                                     double *__restrict__ loss,
                                                     double *__restrict__ grad) {
    const int32_t b = blockIdx.x;
    const size_t o = (size_t)b * n;
    double v[1] = {0.0};
    for (int32_t a = threadIdx.x; a < n; a += kBlock) {
        const double dw = ws[o + a] - wt[o + a];
        v[0] += 2.0 * ch[o + a] * dw + ct[o + a] * wt[o + a];
        grad[o + a] = 2.0 * dw;
    }
    block_sum_all<1>(v);
    if (threadIdx.x == 0) loss[b] = v[0] - zs[b];
}

// Perturbed Fenchel-Young (Berthet et al.), minimisation form: sample (b, m)
// has costs c_hat_b + eps Z_bm; entry i of the [B][M][n] output. Rounded as
// a product then a sum, so the costs equal the textbook expression exactly.
__global__ __launch_bounds__(kBlock) void k_pfy_costs(int64_t N, int32_t M, int32_t n,
                                                      const double *__restrict__ ch,
                                                      const double *__restrict__ Z, double eps,
                                                      double *__restrict__ out) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    const int64_t a = i % n, b = i / n / M;
    const double pz = eps * Z[i];
    out[i] = ch[b * n + a] + pz;
}

// One workgroup per instance: with w_m optimal under c_hat + eps Z_m,
// grad = w* - (1/M) sum_m w_m and loss = c_hat'w* - (1/M) sum_m (c_hat +
// eps Z_m)'w_m (the loss up to the constant Omega(w*)); samples summed in m
// order per variable.
__global__ __launch_bounds__(kBlock) void k_pfy(int32_t M, int32_t n, const double *__restrict__ ch,
                                                const double *__restrict__ ws,
                                                const double *__restrict__ Z, double eps,
                                                const double *__restrict__ wm,
                                                double *__restrict__ loss,
                                                double *__restrict__ grad) {
    const int32_t b = blockIdx.x;
    const size_t o = (size_t)b * n;
    const double dm = (double)M;
    double v[1] = {0.0};
    for (int32_t a = threadIdx.x; a < n; a += kBlock) {
        const double c = ch[o + a];
        double wsum = 0.0, acc = 0.0;
        for (int32_t m = 0; m < M; ++m) {
            const size_t e = ((size_t)b * M + m) * n + a;
            const double w = wm[e];
            wsum += w;
            acc += (c + eps * Z[e]) * w;
        }
        grad[o + a] = ws[o + a] - wsum / dm;
        v[0] += c * ws[o + a] - acc / dm;
    }
    block_sum_all<1>(v);
    if (threadIdx.x == 0) loss[b] = v[0];
}

static unsigned grid1(int64_t N) { return (unsigned)std::max<int64_t>(1, ceil_div(N, kBlock)); }

void head_linear_costs(hipStream_t s, int32_t B, int32_t n, int32_t p, const double *f,
                       const double *W, double *c) {
    const int64_t N = (int64_t)B * n;
    if (N == 0) return;
    k_linear_costs<<<grid1(N), kBlock, 0, s>>>(N, p, f, W, c);
    PDHG_HIP(hipGetLastError());
}

void head_regret(hipStream_t s, int32_t B, int32_t n, const double *ct, const double *x,
                 const double *vs, double *loss) {
    if (B == 0) return;
    k_regret<<<(unsigned)B, kBlock, 0, s>>>(n, ct, x, vs, loss);
    PDHG_HIP(hipGetLastError());
}

void head_linear_costs_backward(hipStream_t s, int32_t B, int32_t n, int32_t p, const double *f,
                                const double *gc, double *gW) {
    const int64_t N = (int64_t)B * n;
    DBuf<double> part;
    part.alloc((size_t)p * kHeadChunks);
    k_costs_grad_part<<<(unsigned)(p * kHeadChunks), kBlock, 0, s>>>(N, p, f, gc, part.p);
    k_costs_grad_final<<<1, 64, 0, s>>>(p, part.p, gW);
    PDHG_HIP(hipGetLastError());
    PDHG_HIP(hipStreamSynchronize(s));
}

// Device address of `scratch` on the device that runs stream s (the current
// device for the NULL stream), looked up once per device with that device
// current.
static double *scratch_address(hipStream_t s) {
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int cur = 0, dev = 0;
    PDHG_HIP(hipGetDevice(&cur));
    dev = cur;
    if (s) PDHG_HIP(hipStreamGetDevice(s, &dev));
    if (dev < 0 || dev >= kMaxDevices) fail(PDHG_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        if (dev != cur) PDHG_HIP(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) PDHG_HIP(hipSetDevice(cur));
        if (e != hipSuccess || !p)
            fail(PDHG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        addr[dev] = static_cast<double *>(p);
    }
    return addr[dev];
}

// The same reduction as head_linear_costs_backward into the static scratch
// array: no allocation and no wait; calls that overlap on one GPU race on it.
void head_linear_costs_backward_noalloc(hipStream_t s, int32_t B, int32_t n, int32_t p,
                                        const double *f, const double *gc, double *gW) {
    if (p < 1 || p > kHeadPmax) fail(PDHG_ERR_INVALID_ARG, "need 1 <= p <= 64 (the scratch holds 64 x 64 partials)");
    const int64_t N = (int64_t)B * n;
    double *part = scratch_address(s);
    k_costs_grad_part<<<(unsigned)(p * kHeadChunks), kBlock, 0, s>>>(N, p, f, gc, part);
    k_costs_grad_final<<<1, 64, 0, s>>>(p, part, gW);
    PDHG_HIP(hipGetLastError());
}

void head_qp_value(hipStream_t s, int32_t B, int32_t n, int32_t r, const double *F,
                   const double *d, const double *c, const double *x, double *value, double *gx) {
    if (B == 0) return;
    if (r > kHeadRmax) fail(PDHG_ERR_UNSUPPORTED, "factor rank above 32");
    k_qp_value<<<(unsigned)B, kBlock, 0, s>>>(n, r, F, d, c, x, value, gx);
    PDHG_HIP(hipGetLastError());
}

void head_spo_costs(hipStream_t s, int32_t B, int32_t n, const double *c_hat, const double *c_true,
                    double *out) {
    const int64_t N = (int64_t)B * n;
    if (N == 0) return;
    k_spo_costs<<<grid1(N), kBlock, 0, s>>>(N, c_hat, c_true, out);
    PDHG_HIP(hipGetLastError());
}

void head_spo_plus(hipStream_t s, int32_t B, int32_t n, const double *c_hat, const double *c_true,
                   const double *w_star, const double *z_star, const double *w_tilde, double *loss,
                   double *grad) {
    if (B == 0) return;
    k_spo_plus<<<(unsigned)B, kBlock, 0, s>>>(n, c_hat, c_true, w_star, z_star, w_tilde, loss, grad);
    PDHG_HIP(hipGetLastError());
}

void head_pfy_costs(hipStream_t s, int32_t B, int32_t M, int32_t n, const double *c_hat,
                    const double *Z, double eps, double *out) {
    const int64_t N = (int64_t)B * M * n;
    if (N == 0) return;
    k_pfy_costs<<<grid1(N), kBlock, 0, s>>>(N, M, n, c_hat, Z, eps, out);
    PDHG_HIP(hipGetLastError());
}

void head_pfy(hipStream_t s, int32_t B, int32_t M, int32_t n, const double *c_hat,
              const double *w_star, const double *Z, double eps, const double *w_samples, double *loss,
              double *grad) {
    if (B == 0) return;
    k_pfy<<<(unsigned)B, kBlock, 0, s>>>(M, n, c_hat, w_star, Z, eps, w_samples, loss, grad);
    PDHG_HIP(hipGetLastError());
}

}  // namespace pdhg
