// Setup on the device: validation, the length-binned internal layout of A and
// A', the diagonal preconditioning of the MPAX paper's Section 3 (Ruiz
// equilibration, then one Pock-Chambolle step with alpha = 1), the power
// iteration for ||A~||_2 that sets the step size, and the initial primal
// weight.
#include <algorithm>
#include <cstring>
#include <exception>
#include <thread>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "device.hpp"

namespace pdhg {

// ---------------------------------------------------------------------------
// validation

__global__ __launch_bounds__(kBlock) void k_validate_rowptr(const int32_t *__restrict__ rowptr,
                                                            int32_t m, int64_t nnz,
                                                            uint8_t *__restrict__ rowstart,
                                                            int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i > m) return;
    const int32_t a = rowptr[i];
    if (i == 0 && a != 0) atomicOr(flag, 1);
    if (i == m) {
        if ((int64_t)a != nnz) atomicOr(flag, 1);
        return;
    }
    const int32_t b = rowptr[i + 1];
    if (b < a || a < 0 || (int64_t)b > nnz) {
        atomicOr(flag, 1);
        return;
    }
    if (b > a) rowstart[a] = 1;
}

__global__ __launch_bounds__(kBlock) void k_validate_entries(const int32_t *__restrict__ colidx,
                                                             const double *__restrict__ val,
                                                             int64_t nnz, int32_t n,
                                                             const uint8_t *__restrict__ rowstart,
                                                             int32_t *__restrict__ flag) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= nnz) return;
    const int32_t j = colidx[e];
    if (j < 0 || j >= n || !isfinite(val[e])) atomicOr(flag, 2);
    if (e + 1 < nnz && !rowstart[e + 1] && colidx[e + 1] <= j) atomicOr(flag, 4);
}

// c finite; l <= u, no NaN, l != +inf, u != -inf.
__global__ __launch_bounds__(kBlock) void k_validate_vectors(int32_t n, int32_t m,
                                                             const double *__restrict__ c,
                                                             const double *__restrict__ lv,
                                                             const double *__restrict__ uv,
                                                             const double *__restrict__ lc,
                                                             const double *__restrict__ uc,
                                                             int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double l = lv[i], u = uv[i];
        if (!isfinite(c[i]) || isnan(l) || isnan(u) || l > u || l == INFINITY || u == -INFINITY)
            atomicOr(flag, 8);
    } else if (i - n < m) {
        const int64_t r = i - n;
        const double l = lc[r], u = uc[r];
        if (isnan(l) || isnan(u) || l > u || l == INFINITY || u == -INFINITY) atomicOr(flag, 16);
    }
}

// ---------------------------------------------------------------------------
// length classes and the internal layout

// Sort key: descending exact length (ascending key).
__global__ __launch_bounds__(kBlock) void k_row_keys(const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ cnt, int32_t len,
                                                     uint32_t kmax, uint32_t *__restrict__ key,
                                                     int32_t *__restrict__ iota) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= len) return;
    const int32_t l = rowptr ? rowptr[i + 1] - rowptr[i] : cnt[i];
    key[i] = kmax - (uint32_t)l;
    iota[i] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_col_count(const int32_t *__restrict__ colidx,
                                                      int64_t nnz, int32_t *__restrict__ cnt) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < nnz) atomicAdd(&cnt[colidx[e]], 1);
}

__global__ __launch_bounds__(kBlock) void k_inverse(const int32_t *__restrict__ perm, int32_t len,
                                                    int32_t *__restrict__ inv) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) inv[perm[i]] = (int32_t)i;
}

// first[j] = smallest internal row index among the entries of original column
// j (one thread per original row; first[] starts at INT32_MAX).
__global__ __launch_bounds__(kBlock) void k_first_row(const int32_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ colidx,
                                                      const int32_t *__restrict__ inv_r, int32_t m,
                                                      int32_t *__restrict__ first) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    const int32_t ir = inv_r[i];
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) atomicMin(&first[colidx[e]], ir);
}

// len_int[i'] = length of original row perm[i'] (rowptr form or count form);
// len_int[len] = 0 so that an exclusive scan gives the full rowptr.
__global__ __launch_bounds__(kBlock) void k_perm_lengths(const int32_t *__restrict__ perm,
                                                         const int32_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ counts,
                                                         int32_t len, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i > len) return;
    if (i == len) {
        out[i] = 0;
        return;
    }
    const int32_t r = perm[i];
    out[i] = rowptr ? rowptr[r + 1] - rowptr[r] : counts[r];
}

// One wave per internal row: copy the original row with relabelled columns.
__global__ __launch_bounds__(kBlock) void k_fill_internal(
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const double *__restrict__ val, const int32_t *__restrict__ perm_r,
    const int32_t *__restrict__ inv_c, const int32_t *__restrict__ rp_int, int32_t m,
    int32_t *__restrict__ ci_int, double *__restrict__ va_int, int32_t *__restrict__ row_of) {
    const int64_t w = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= m) return;
    const int32_t src = perm_r[w];
    const int32_t s0 = rowptr[src], s1 = rowptr[src + 1];
    const int32_t d0 = rp_int[w];
    for (int32_t e = s0 + lane; e < s1; e += 64) {
        const int32_t d = d0 + (e - s0);
        ci_int[d] = inv_c[colidx[e]];
        va_int[d] = val[e];
        row_of[d] = (int32_t)w;
    }
}

// row id of every entry of a plain CSR (one wave per row)
__global__ __launch_bounds__(kBlock) void k_row_of(const int32_t *__restrict__ rowptr, int32_t rows,
                                                   int32_t *__restrict__ row_of) {
    const int64_t w = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= rows) return;
    for (int32_t e = rowptr[w] + lane; e < rowptr[w + 1]; e += 64) row_of[e] = (int32_t)w;
}

__global__ __launch_bounds__(kBlock) void k_iota_u(int32_t *__restrict__ iota, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) iota[i] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_fill_transpose(const int32_t *__restrict__ order,
                                                           const int32_t *__restrict__ row_of,
                                                           const double *__restrict__ va,
                                                           int64_t nnz, int32_t *__restrict__ ci_t,
                                                           double *__restrict__ va_t) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= nnz) return;
    const int32_t e = order[p];
    ci_t[p] = row_of[e];
    va_t[p] = va[e];
}

// Number of leading rows longer than the short-row limit (rows sorted by
// descending length) and the length histogram of those rows by class
// (class c >= 1: length in (2^(c-1), 2^c]).
__global__ __launch_bounds__(kBlock) void k_long_rows(const int32_t *__restrict__ rowptr,
                                                      int32_t rows, int32_t limit,
                                                      int32_t *__restrict__ out /*[1+32]*/) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= rows) return;
    const int32_t l = rowptr[i + 1] - rowptr[i];
    if (l > limit) {
        const int32_t nl = (i + 1 < rows) ? rowptr[i + 2] - rowptr[i + 1] : 0;
        if (nl <= limit) out[0] = (int32_t)(i + 1);
        const int32_t cls = 32 - __clz(l - 1);
        atomicAdd(&out[1 + (31 - cls)], 1);
    }
}

// widths64[s] = 64 * length of the first row of slice s; widths64[ns] = 0.
__global__ __launch_bounds__(kBlock) void k_slice_widths(const int32_t *__restrict__ rowptr,
                                                         int32_t r_long, int32_t ns,
                                                         int32_t *__restrict__ widths64) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s > ns) return;
    if (s == ns) {
        widths64[s] = 0;
        return;
    }
    const int64_t r = r_long + s * 64;
    widths64[s] = 64 * (rowptr[r + 1] - rowptr[r]);
}

__global__ __launch_bounds__(kBlock) void k_add_offset(const int32_t *__restrict__ in, int32_t len,
                                                       int32_t off, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) out[i] = in[i] + off;
}

// Copy the short rows into their SELL-64 slices, padding with (0, 0.0).
__global__ __launch_bounds__(kBlock) void k_fill_slices(const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ colidx,
                                                        const double *__restrict__ val,
                                                        int32_t r_long, int32_t rows, int32_t ns,
                                                        const int32_t *__restrict__ slice_ptr,
                                                        int32_t *__restrict__ ci_out,
                                                        double *__restrict__ va_out) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t s = t >> 6;
    const int32_t lane = (int32_t)(t & 63);
    if (s >= ns) return;
    const int64_t r = r_long + s * 64 + lane;
    const int32_t b = slice_ptr[s];
    const int32_t w = (slice_ptr[s + 1] - b) >> 6;
    const int32_t e0 = r < rows ? rowptr[r] : 0;
    const int32_t len = r < rows ? rowptr[r + 1] - e0 : 0;
    for (int32_t k = 0; k < w; ++k) {
        const int32_t d = b + 64 * k + lane;
        ci_out[d] = k < len ? colidx[e0 + k] : 0;
        va_out[d] = k < len ? val[e0 + k] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// scaling kernels

template <bool MAXNORM>
__global__ __launch_bounds__(kBlock) void k_row_absnorm(MatView M, double *__restrict__ out) {
    const RowSum rs = mat_row_absnorm<MAXNORM>(M);
    if (rs.valid) out[rs.row] = rs.s;
}

// factor f = sqrt(norm) (1 for an empty row / column); D <- D / f.
__global__ __launch_bounds__(kBlock) void k_factors(double *__restrict__ norm_to_factor,
                                                    double *__restrict__ D, int32_t len) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= len) return;
    const double v = norm_to_factor[i];
    const double f = v > 0.0 ? sqrt(v) : 1.0;
    norm_to_factor[i] = f;
    D[i] = D[i] / f;
}

// A~_ij <- A~_ij / (r_i s_j) for the rows of A (transposed = 0) or of A'.
__global__ __launch_bounds__(kBlock) void k_scale_vals(MatView M, const double *__restrict__ rfac,
                                                       const double *__restrict__ cfac,
                                                       int32_t transposed) {
    mat_scale_entries(M, rfac, cfac, transposed != 0);
}

// c~ = D_c c, l~_v = l_v / D_c, u~_v = u_v / D_c (columns); l~_c = D_r l_c,
// u~_c = D_r u_c (rows).
__global__ __launch_bounds__(kBlock) void k_transform(
    int32_t n, int32_t m, const double *__restrict__ Dc, const double *__restrict__ Dr,
    const double *__restrict__ c_o, const double *__restrict__ lv_o,
    const double *__restrict__ uv_o, const double *__restrict__ lc_o,
    const double *__restrict__ uc_o, double *__restrict__ c, double *__restrict__ lv,
    double *__restrict__ uv, double *__restrict__ lc, double *__restrict__ uc) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double d = Dc[i];
        c[i] = d * c_o[i];
        lv[i] = lv_o[i] / d;
        uv[i] = uv_o[i] / d;
    } else if (i - n < m) {
        const int64_t r = i - n;
        const double d = Dr[r];
        lc[r] = d * lc_o[r];
        uc[r] = d * uc_o[r];
    }
}

__global__ __launch_bounds__(kBlock) void k_fill(double *__restrict__ v, double value, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) v[i] = value;
}

// Sums for the norms: 0 |c~|^2, 1 |b~|^2 (scaled), 2 |c|^2, 3 |b|^2 (original),
// with b_i the largest finite |bound| of row i.
__global__ __launch_bounds__(kBlock) void k_norm_sums(int32_t n, int32_t m,
                                                      const double *__restrict__ c,
                                                      const double *__restrict__ lc,
                                                      const double *__restrict__ uc,
                                                      const double *__restrict__ c_o,
                                                      const double *__restrict__ lc_o,
                                                      const double *__restrict__ uc_o,
                                                      double *__restrict__ partials) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)n + m; i += stride) {
        if (i < n) {
            v[0] += c[i] * c[i];
            v[2] += c_o[i] * c_o[i];
        } else {
            const int64_t r = i - n;
            double b = 0.0, bo = 0.0;
            if (isfinite(lc[r])) b = fmax(b, fabs(lc[r]));
            if (isfinite(uc[r])) b = fmax(b, fabs(uc[r]));
            if (isfinite(lc_o[r])) bo = fmax(bo, fabs(lc_o[r]));
            if (isfinite(uc_o[r])) bo = fmax(bo, fabs(uc_o[r]));
            v[1] += b * b;
            v[3] += bo * bo;
        }
    }
    block_sum_store<4>(v, partials + (size_t)blockIdx.x * 4);
}

// out = A~ v on the rows of a matrix, partial sums of out^2.
__global__ __launch_bounds__(kBlock) void k_spmv_sq(MatView M, const double *__restrict__ v,
                                                    double *__restrict__ out,
                                                    double *__restrict__ partials) {
    const RowSum rs = mat_row_dot(M, v);
    double q[1] = {0.0};
    if (rs.valid) {
        out[rs.row] = rs.s;
        q[0] = rs.s * rs.s;
    }
    block_sum_store<1>(q, partials + blockIdx.x);
}

// Start vector of the power iteration: v_j = 0.5 + u_j with u_j uniform in
// [0, 1) from SplitMix64 (Steele, Lea and Flood, 2014) at counter j, j the
// ORIGINAL column index; also partial sums of v^2.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_power_start(const int32_t *__restrict__ perm_c, int32_t n,
                                                        double *__restrict__ v,
                                                        double *__restrict__ partials) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double q[1] = {0.0};
    if (i < n) {
        const double u = (double)(splitmix64((uint64_t)perm_c[i]) >> 11) * 0x1.0p-53;
        const double val = 0.5 + u;
        v[i] = val;
        q[0] = val * val;
    }
    block_sum_store<1>(q, partials + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_div_sqrt(double *__restrict__ v, int32_t n,
                                                     const double *__restrict__ tot) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) v[i] = v[i] / sqrt(tot[0]);
}

// Fixed-order total of K-wide partials, written to out[0..K-1].
template <int K>
__global__ __launch_bounds__(kBlock) void k_total(const double *__restrict__ partials, int32_t nb,
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

// v = u / |u|, |u|^2 = tot[0]; records lam (= |A~ v_prev|^2 = wtot[0]) and |u|.
__global__ __launch_bounds__(kBlock) void k_power_normalize(const double *__restrict__ u,
                                                            double *__restrict__ v, int32_t n,
                                                            const double *__restrict__ wtot,
                                                            const double *__restrict__ utot,
                                                            double *__restrict__ hist, int32_t it) {
    const double nu = sqrt(utot[0]);
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) {
        hist[2 * it] = wtot[0];
        hist[2 * it + 1] = nu;
    }
    if (i < n && nu > 0.0) v[i] = u[i] / nu;
}

// Golub-Kahan-Lanczos step pieces. w <- w - coef[0] prev (coef a device
// scalar), with per-workgroup partial sums of w^2.
__global__ __launch_bounds__(kBlock) void k_lanczos_sub(double *__restrict__ w,
                                                        const double *__restrict__ prev,
                                                        const double *__restrict__ coef, int32_t len,
                                                        double *__restrict__ partials) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double q[1] = {0.0};
    if (i < len) {
        const double r = w[i] - coef[0] * prev[i];
        w[i] = r;
        q[0] = r * r;
    }
    block_sum_store<1>(q, partials + blockIdx.x);
}

// out = w / |w| with |w|^2 = tot[0]; records |w| in *slot.
__global__ __launch_bounds__(kBlock) void k_lanczos_scale(const double *__restrict__ w,
                                                          double *__restrict__ out, int32_t len,
                                                          const double *__restrict__ tot,
                                                          double *__restrict__ slot) {
    const double nw = sqrt(tot[0]);
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) slot[0] = nw;
    if (i < len && nw > 0.0) out[i] = w[i] / nw;
}

// ---------------------------------------------------------------------------
// host side

namespace {

template <class F>
void with_temp(hipStream_t s, F &&f) {
    size_t bytes = 0;
    PDHG_HIP(f(nullptr, bytes));
    DBuf<uint8_t> tmp;
    tmp.alloc(bytes);
    PDHG_HIP(f(tmp.p, bytes));
    (void)s;
}

void sort_pairs(hipStream_t s, const uint32_t *kin, uint32_t *kout, const int32_t *vin,
                int32_t *vout, int64_t len, int bits) {
    if (len <= 0) return;
    with_temp(s, [&](void *tmp, size_t &bytes) {
        return rocprim::radix_sort_pairs(tmp, bytes, kin, kout, vin, vout, (size_t)len, 0u,
                                         (unsigned)bits, s);
    });
}

void exclusive_scan(hipStream_t s, const int32_t *in, int32_t *out, int64_t len) {
    with_temp(s, [&](void *tmp, size_t &bytes) {
        return rocprim::exclusive_scan(tmp, bytes, in, out, 0, (size_t)len,
                                       rocprim::plus<int32_t>(), s);
    });
}

unsigned blocks_for(int64_t len) { return (unsigned)std::max<int64_t>(1, ceil_div(len, kBlock)); }

}  // namespace

SegTable make_segments(const std::vector<int32_t> &class_count, int32_t rows) {
    SegTable T;
    memset(&T, 0, sizeof(T));
    int32_t begin = 0, blocks = 0;
    for (int q = 0; q < 32; ++q) {
        const int32_t cnt = class_count[q];
        if (cnt <= 0) continue;
        const int cls = 31 - q;
        const int lg = std::min(6, std::max(0, cls - 2));
        const int32_t rows_per_block = kBlock >> lg;
        Seg sg;
        sg.row_begin = begin;
        sg.row_end = begin + cnt;
        sg.lanes_log2 = lg;
        sg.block_begin = blocks;
        T.s[T.nseg++] = sg;
        begin += cnt;
        blocks += (int32_t)ceil_div(cnt, rows_per_block);
    }
    if (begin != rows) fail(PDHG_ERR_INVALID_INPUT, "internal: class counts do not add up");
    T.nblocks = blocks;
    return T;
}

void check_flag(hipStream_t s, const int32_t *dflag, const char *what) {
    int32_t f = 0;
    PDHG_HIP(hipMemcpyAsync(&f, dflag, sizeof(f), hipMemcpyDeviceToHost, s));
    PDHG_HIP(hipStreamSynchronize(s));
    if (f) fail(PDHG_ERR_INVALID_INPUT, std::string(what) + " (code " + std::to_string(f) + ")");
}

// Device copy of a caller array (or a view when it already is on the device).
template <class T>
static const T *device_view(const T *src, size_t count, int mem, DBuf<T> &holder, hipStream_t s) {
    if (mem == PDHG_MEM_DEVICE || count == 0) return src;
    holder.alloc(count);
    PDHG_HIP(hipMemcpyAsync(holder.p, src, count * sizeof(T), hipMemcpyHostToDevice, s));
    return holder.p;
}

// Plain CSR in internal order (temporary, before conversion to the hybrid layout).
struct PlainCsr {
    int32_t rows = 0;
    int64_t nnz = 0;
    DBuf<int32_t> rowptr, colidx;
    DBuf<double> val;
};

// Convert a plain CSR whose rows are sorted by descending length into the
// hybrid layout (long rows as CSR with lane groups, the rest as SELL-64).
static void to_hybrid(hipStream_t s, PlainCsr &P, int32_t cols, HMat &H) {
    const int32_t R = P.rows;
    H.rows = R;
    H.cols = cols;
    H.nnz = P.nnz;
    DBuf<int32_t> info;
    info.alloc(33);
    PDHG_HIP(hipMemsetAsync(info.p, 0, 33 * sizeof(int32_t), s));
    if (R > 0) k_long_rows<<<blocks_for(R), kBlock, 0, s>>>(P.rowptr.p, R, kShortMax, info.p);
    int32_t hinfo[33];
    PDHG_HIP(hipMemcpyAsync(hinfo, info.p, sizeof(hinfo), hipMemcpyDeviceToHost, s));
    PDHG_HIP(hipStreamSynchronize(s));
    const int32_t r_long = hinfo[0];
    std::vector<int32_t> cls(hinfo + 1, hinfo + 33);
    H.R_long = r_long;
    H.seg = make_segments(cls, r_long);
    const int32_t ns = (int32_t)ceil_div(R - r_long, 64);
    H.nslices = ns;
    int32_t nnz_long = 0;
    if (r_long > 0)
        PDHG_HIP(hipMemcpyAsync(&nnz_long, P.rowptr.p + r_long, sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
    DBuf<int32_t> widths, soff;
    widths.alloc((size_t)ns + 1);
    soff.alloc((size_t)ns + 1);
    k_slice_widths<<<blocks_for((int64_t)ns + 1), kBlock, 0, s>>>(P.rowptr.p, r_long, ns, widths.p);
    exclusive_scan(s, widths.p, soff.p, (int64_t)ns + 1);
    int32_t short_total = 0;
    PDHG_HIP(hipMemcpyAsync(&short_total, soff.p + ns, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PDHG_HIP(hipStreamSynchronize(s));
    if ((int64_t)nnz_long + short_total >= INT32_MAX)
        fail(PDHG_ERR_UNSUPPORTED, "matrix too large for 32-bit entry offsets after padding");
    H.stored = (int64_t)nnz_long + short_total;
    H.colidx.alloc((size_t)H.stored);
    H.val.alloc((size_t)H.stored);
    H.rowptr.alloc((size_t)r_long + 1);
    H.slice_ptr.alloc((size_t)ns + 1);
    PDHG_HIP(hipMemcpyAsync(H.rowptr.p, P.rowptr.p, sizeof(int32_t) * ((size_t)r_long + 1),
                            hipMemcpyDeviceToDevice, s));
    if (nnz_long > 0) {
        PDHG_HIP(hipMemcpyAsync(H.colidx.p, P.colidx.p, sizeof(int32_t) * (size_t)nnz_long,
                                hipMemcpyDeviceToDevice, s));
        PDHG_HIP(hipMemcpyAsync(H.val.p, P.val.p, sizeof(double) * (size_t)nnz_long,
                                hipMemcpyDeviceToDevice, s));
    }
    k_add_offset<<<blocks_for((int64_t)ns + 1), kBlock, 0, s>>>(soff.p, ns + 1, nnz_long,
                                                                H.slice_ptr.p);
    if (ns > 0)
        k_fill_slices<<<blocks_for((int64_t)ns * 64), kBlock, 0, s>>>(
            P.rowptr.p, P.colidx.p, P.val.p, r_long, R, ns, H.slice_ptr.p, H.colidx.p, H.val.p);
    PDHG_HIP(hipStreamSynchronize(s));
}

void validate_csr(hipStream_t s, const int32_t *rowptr, const int32_t *colidx,
                  const double *val, int32_t m, int32_t n, int64_t nnz) {
    DBuf<int32_t> flag;
    flag.alloc(1);
    PDHG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    DBuf<uint8_t> rowstart;
    rowstart.alloc((size_t)nnz + 1);
    PDHG_HIP(hipMemsetAsync(rowstart.p, 0, (size_t)nnz + 1, s));
    k_validate_rowptr<<<blocks_for((int64_t)m + 1), kBlock, 0, s>>>(rowptr, m, nnz, rowstart.p,
                                                                     flag.p);
    check_flag(s, flag.p, "invalid CSR row pointers");
    if (nnz > 0)
        k_validate_entries<<<blocks_for(nnz), kBlock, 0, s>>>(colidx, val, nnz, n, rowstart.p,
                                                               flag.p);
    check_flag(s, flag.p, "invalid CSR entries (column out of range, unsorted or duplicate "
                          "column, or non-finite value)");
}

void validate_vectors(hipStream_t s, int32_t n, int32_t m, const double *c, const double *lv,
                      const double *uv, const double *lc, const double *uc) {
    DBuf<int32_t> flag;
    flag.alloc(1);
    PDHG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    k_validate_vectors<<<blocks_for((int64_t)n + m), kBlock, 0, s>>>(n, m, c, lv, uv, lc, uc,
                                                                    flag.p);
    check_flag(s, flag.p, "invalid objective or bounds (non-finite c, NaN bound, l > u)");
}

void plain_transpose(hipStream_t s, int32_t rows, int32_t cols, int64_t nnz,
                     const int32_t *rowptr, const int32_t *colidx, const double *val,
                     int32_t *rowptr_t, int32_t *colidx_t, double *val_t) {
    DBuf<int32_t> cnt, row_of;
    cnt.alloc((size_t)cols + 1);
    PDHG_HIP(hipMemsetAsync(cnt.p, 0, ((size_t)cols + 1) * sizeof(int32_t), s));
    if (nnz > 0) k_col_count<<<blocks_for(nnz), kBlock, 0, s>>>(colidx, nnz, cnt.p);
    exclusive_scan(s, cnt.p, rowptr_t, (int64_t)cols + 1);
    if (nnz == 0) return;
    row_of.alloc((size_t)nnz);
    if (rows > 0) k_row_of<<<blocks_for((int64_t)rows * 64), kBlock, 0, s>>>(rowptr, rows, row_of.p);
    DBuf<uint32_t> ekey_sorted;
    DBuf<int32_t> eid, order;
    ekey_sorted.alloc((size_t)nnz);
    eid.alloc((size_t)nnz);
    order.alloc((size_t)nnz);
    k_iota_u<<<blocks_for(nnz), kBlock, 0, s>>>(eid.p, nnz);
    int bits = 1;
    while ((1ll << bits) < (int64_t)cols) ++bits;
    sort_pairs(s, reinterpret_cast<const uint32_t *>(colidx), ekey_sorted.p, eid.p, order.p, nnz,
               bits);
    k_fill_transpose<<<blocks_for(nnz), kBlock, 0, s>>>(order.p, row_of.p, val, nnz, colidx_t,
                                                        val_t);
    PDHG_HIP(hipStreamSynchronize(s));
}

void permute_csr(hipStream_t s, int32_t rows, int32_t cols, int64_t nnz, const int32_t *rowptr,
                 const int32_t *colidx, const double *val, const int32_t *perm_r,
                 const int32_t *perm_c, int32_t *out_rp, int32_t *out_ci, double *out_va) {
    DBuf<int32_t> inv_c, lens, row_of;
    inv_c.alloc(cols);
    k_inverse<<<blocks_for(cols), kBlock, 0, s>>>(perm_c, cols, inv_c.p);
    lens.alloc((size_t)rows + 1);
    k_perm_lengths<<<blocks_for((int64_t)rows + 1), kBlock, 0, s>>>(perm_r, rowptr, nullptr, rows,
                                                                    lens.p);
    exclusive_scan(s, lens.p, out_rp, (int64_t)rows + 1);
    row_of.alloc((size_t)nnz);
    if (rows > 0 && nnz > 0)
        k_fill_internal<<<blocks_for((int64_t)rows * 64), kBlock, 0, s>>>(
            rowptr, colidx, val, perm_r, inv_c.p, out_rp, rows, out_ci, out_va, row_of.p);
    PDHG_HIP(hipStreamSynchronize(s));
}

// Rows of y per LDS panel of the primal product (0: the panels are off).
static int32_t panel_rows(const pdhg_options &o, int32_t m) {
    if (o.panel_rows == 0) return 0;
    if (o.panel_rows > 0) return o.panel_rows;
    return m > 262144 ? kPanelMax : 0;
}

// With the LDS panels in use, the columns of A that k_primal_sell runs (the
// SELL-64 rows of A~' from R on, R as keep_panel_rows sets it) are reordered
// within each length: k_primal_sell's workgroup w takes 256 consecutive of
// them and runs on XCD w mod 8, so the columns whose first entry (smallest
// internal row) falls in eighth e of y go where (w mod 8) = e, as far as each
// length has such columns. One of the entries a workgroup gathers per column
// then lies in the eighth of y that its XCD keeps reading (an L2-sized
// window). Any column order is valid: this only changes which L2 serves a
// gather.
static void interleave_short_columns(Handle &h, hipStream_t s, const int32_t *rowptr, const int32_t *colidx,
                                     const int32_t *cnt, int32_t m, int32_t n) {
    if (m < 8 || n < 1) return;
    DBuf<int32_t> inv_r, first;
    inv_r.alloc(m);
    first.alloc(n);
    k_inverse<<<blocks_for(m), kBlock, 0, s>>>(h.perm_r.p, m, inv_r.p);
    std::vector<int32_t> init((size_t)n, INT32_MAX);
    PDHG_HIP(hipMemcpyAsync(first.p, init.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    k_first_row<<<blocks_for(m), kBlock, 0, s>>>(rowptr, colidx, inv_r.p, m, first.p);
    std::vector<int32_t> perm((size_t)n), len((size_t)n), fr((size_t)n);
    PDHG_HIP(hipMemcpyAsync(perm.data(), h.perm_c.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    PDHG_HIP(hipMemcpyAsync(len.data(), cnt, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    PDHG_HIP(hipMemcpyAsync(fr.data(), first.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    PDHG_HIP(hipStreamSynchronize(s));
    // R: the first row of A~' that k_primal_sell runs (the hybrid layout's
    // R_long, then the panel rows up to a whole slice)
    auto L = [&](int32_t q) { return len[(size_t)perm[(size_t)q]]; };
    const int32_t min_len = h.opt.panel_min_len < 0 ? 32 : h.opt.panel_min_len;
    int32_t rl = 0, rt = 0;
    while (rl < n && L(rl) > kShortMax) ++rl;
    while (rt < n && L(rt) > min_len) ++rt;
    int32_t R = rl;
    if (rt > rl) R = (int32_t)std::min<int64_t>(n, rl + 64 * ceil_div(rt - rl, 64));
    const int32_t win = (m + 7) / 8;
    constexpr int32_t kCols = kBlock;   // columns per workgroup of k_primal_sell
    std::vector<int32_t> q[8];
    for (int32_t a = R; a < n;) {
        int32_t b = a;
        while (b < n && L(b) == L(a)) ++b;
        for (auto &v : q) v.clear();
        for (int32_t t = a; t < b; ++t) {
            const int32_t j = perm[(size_t)t];
            const int32_t f = fr[(size_t)j];
            q[f == INT32_MAX ? 7 : std::min(7, f / win)].push_back(j);
        }
        size_t head[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int32_t t = a; t < b; ++t) {
            int32_t e = ((t - R) / kCols) % 8;
            for (int k = 0; k < 8 && head[e] == q[e].size(); ++k) e = (e + 1) % 8;
            perm[(size_t)t] = q[e][head[e]++];
        }
        a = b;
    }
    PDHG_HIP(hipMemcpyAsync(h.perm_c.p, perm.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    PDHG_HIP(hipStreamSynchronize(s));
}

// Choose the rows of A~' that the LDS panels cover: the rows longer than
// panel_min_len, extended to whole SELL-64 slices (rows are sorted by length,
// the first R_long of them stored as CSR). Their structure is kept on the host
// until the scaled values exist.
static void keep_panel_rows(Handle &h, const PlainCsr &PT, int32_t m) {
    const int32_t n = PT.rows;
    const int32_t S = panel_rows(h.opt, m);
    if (S <= 0 || m <= 0 || PT.nnz == 0) return;
    std::vector<int32_t> rp((size_t)n + 1);
    PDHG_HIP(hipMemcpy(rp.data(), PT.rowptr.p, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost));
    const int32_t min_len = h.opt.panel_min_len < 0 ? 32 : h.opt.panel_min_len;
    int32_t rt = 0;
    while (rt < n && rp[rt + 1] - rp[rt] > min_len) ++rt;
    const int32_t RL = h.AT.R_long;
    int32_t R = RL;
    if (rt > RL) R = (int32_t)std::min<int64_t>(n, RL + 64 * ceil_div(rt - RL, 64));
    if (R == 0 || rp[R] == 0) return;
    h.PT.R = R;
    h.PT.S = S;
    h.sell_skip = (int32_t)ceil_div(R - RL, 64);
    rp.resize((size_t)R + 1);
    h.at_colidx_host.resize((size_t)rp[R]);
    PDHG_HIP(hipMemcpy(h.at_colidx_host.data(), PT.colidx.p, sizeof(int32_t) * (size_t)rp[R],
                       hipMemcpyDeviceToHost));
    h.at_rowptr_host = std::move(rp);
}

void build_matrices(Handle &h, const pdhg_problem &p) {
    hipStream_t s = h.stream;
    const int32_t m = p.m, n = p.n;
    const int64_t nnz = p.a_nnz;
    DBuf<int32_t> hrp, hci;
    DBuf<double> hva;
    const int32_t *rowptr = device_view(p.a_rowptr, (size_t)m + 1, p.mem, hrp, s);
    const int32_t *colidx = device_view(p.a_colidx, (size_t)nnz, p.mem, hci, s);
    const double *val = device_view(p.a_val, (size_t)nnz, p.mem, hva, s);

    DBuf<int32_t> flag;
    flag.alloc(1);
    PDHG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    {
        DBuf<uint8_t> rowstart;
        rowstart.alloc((size_t)nnz + 1);
        PDHG_HIP(hipMemsetAsync(rowstart.p, 0, (size_t)nnz + 1, s));
        k_validate_rowptr<<<blocks_for((int64_t)m + 1), kBlock, 0, s>>>(rowptr, m, nnz,
                                                                         rowstart.p, flag.p);
        check_flag(s, flag.p, "invalid CSR row pointers");
        if (nnz > 0)
            k_validate_entries<<<blocks_for(nnz), kBlock, 0, s>>>(colidx, val, nnz, n, rowstart.p,
                                                                   flag.p);
        check_flag(s, flag.p, "invalid CSR entries (column out of range, unsorted or duplicate "
                              "column, or non-finite value)");
    }

    // permutations by descending exact length (stable)
    h.perm_r.alloc(m);
    h.perm_c.alloc(n);
    int kbits = 1;
    while ((1ll << kbits) <= (int64_t)std::max(m, n) + 1) ++kbits;
    const uint32_t kmax = (uint32_t)((1ull << kbits) - 1);
    {
        DBuf<uint32_t> key, key_sorted;
        DBuf<int32_t> iota, cnt;
        key.alloc(std::max(m, n));
        key_sorted.alloc(std::max(m, n));
        iota.alloc(std::max(m, n));
        cnt.alloc(n);
        if (m > 0) {
            k_row_keys<<<blocks_for(m), kBlock, 0, s>>>(rowptr, nullptr, m, kmax, key.p, iota.p);
            sort_pairs(s, key.p, key_sorted.p, iota.p, h.perm_r.p, m, kbits);
        }
        PDHG_HIP(hipMemsetAsync(cnt.p, 0, (size_t)n * sizeof(int32_t), s));
        if (nnz > 0) k_col_count<<<blocks_for(nnz), kBlock, 0, s>>>(colidx, nnz, cnt.p);
        k_row_keys<<<blocks_for(n), kBlock, 0, s>>>(nullptr, cnt.p, n, kmax, key.p, iota.p);
        sort_pairs(s, key.p, key_sorted.p, iota.p, h.perm_c.p, n, kbits);
        key.release();
        key_sorted.release();
        if (panel_rows(h.opt, m) > 0 && p.q_format == PDHG_FMT_NONE && nnz > 0)
            interleave_short_columns(h, s, rowptr, colidx, cnt.p, m, n);

        DBuf<int32_t> inv_c, lens, row_of;
        inv_c.alloc(n);
        k_inverse<<<blocks_for(n), kBlock, 0, s>>>(h.perm_c.p, n, inv_c.p);

        // plain internal A
        PlainCsr PA;
        PA.rows = m;
        PA.nnz = nnz;
        PA.rowptr.alloc((size_t)m + 1);
        PA.colidx.alloc((size_t)nnz);
        PA.val.alloc((size_t)nnz);
        row_of.alloc((size_t)nnz);
        lens.alloc((size_t)std::max(m, n) + 1);
        k_perm_lengths<<<blocks_for((int64_t)m + 1), kBlock, 0, s>>>(h.perm_r.p, rowptr, nullptr, m,
                                                                     lens.p);
        exclusive_scan(s, lens.p, PA.rowptr.p, (int64_t)m + 1);
        if (m > 0 && nnz > 0)
            k_fill_internal<<<blocks_for((int64_t)m * 64), kBlock, 0, s>>>(
                rowptr, colidx, val, h.perm_r.p, inv_c.p, PA.rowptr.p, m, PA.colidx.p, PA.val.p,
                row_of.p);

        // plain internal A' by a stable sort of the entries on their internal column
        PlainCsr PT;
        PT.rows = n;
        PT.nnz = nnz;
        PT.rowptr.alloc((size_t)n + 1);
        PT.colidx.alloc((size_t)nnz);
        PT.val.alloc((size_t)nnz);
        k_perm_lengths<<<blocks_for((int64_t)n + 1), kBlock, 0, s>>>(h.perm_c.p, nullptr, cnt.p, n,
                                                                     lens.p);
        exclusive_scan(s, lens.p, PT.rowptr.p, (int64_t)n + 1);
        if (nnz > 0) {
            DBuf<uint32_t> ekey_sorted;
            DBuf<int32_t> eid, order;
            ekey_sorted.alloc((size_t)nnz);
            eid.alloc((size_t)nnz);
            order.alloc((size_t)nnz);
            k_iota_u<<<blocks_for(nnz), kBlock, 0, s>>>(eid.p, nnz);
            int bits = 1;
            while ((1ll << bits) < (int64_t)n) ++bits;
            sort_pairs(s, reinterpret_cast<const uint32_t *>(PA.colidx.p), ekey_sorted.p, eid.p,
                       order.p, nnz, bits);
            k_fill_transpose<<<blocks_for(nnz), kBlock, 0, s>>>(order.p, row_of.p, PA.val.p, nnz,
                                                                PT.colidx.p, PT.val.p);
        }
        PDHG_HIP(hipStreamSynchronize(s));
        to_hybrid(s, PA, n, h.A);
        to_hybrid(s, PT, m, h.AT);
        if (p.q_format == PDHG_FMT_NONE) keep_panel_rows(h, PT, m);
    }
    PDHG_HIP(hipStreamSynchronize(s));
}

void validate_and_load_vectors(Handle &h, const pdhg_problem &p) {
    hipStream_t s = h.stream;
    const int32_t m = h.m, n = h.n;
    DBuf<double> hc, hlv, huv, hlc, huc;
    const double *c = device_view(p.c, (size_t)n, p.mem, hc, s);
    const double *lv = device_view(p.lv, (size_t)n, p.mem, hlv, s);
    const double *uv = device_view(p.uv, (size_t)n, p.mem, huv, s);
    const double *lc = device_view(p.lc, (size_t)m, p.mem, hlc, s);
    const double *uc = device_view(p.uc, (size_t)m, p.mem, huc, s);
    DBuf<int32_t> flag;
    flag.alloc(1);
    PDHG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    k_validate_vectors<<<blocks_for((int64_t)n + m), kBlock, 0, s>>>(n, m, c, lv, uv, lc, uc,
                                                                    flag.p);
    check_flag(s, flag.p, "invalid objective or bounds (non-finite c, NaN bound, l > u)");
    for (auto *b : {&h.c_o, &h.lv_o, &h.uv_o, &h.c, &h.lv, &h.uv, &h.Dc, &h.x, &h.x0, &h.xhat,
                    &h.xext, &h.aty})
        if (!b->p) b->alloc(n);
    for (auto *b : {&h.lc_o, &h.uc_o, &h.lc, &h.uc, &h.Dr, &h.y, &h.y0, &h.yhat})
        if (!b->p) b->alloc(m);
    launch_gather(s, h.perm_c.p, c, h.c_o.p, n);
    launch_gather(s, h.perm_c.p, lv, h.lv_o.p, n);
    launch_gather(s, h.perm_c.p, uv, h.uv_o.p, n);
    launch_gather(s, h.perm_r.p, lc, h.lc_o.p, m);
    launch_gather(s, h.perm_r.p, uc, h.uc_o.p, m);
    PDHG_HIP(hipStreamSynchronize(s));
}

void launch_factors(Handle &h, double *rn, double *cn) {
    if (h.m > 0) k_factors<<<blocks_for(h.m), kBlock, 0, h.stream>>>(rn, h.Dr.p, h.m);
    k_factors<<<blocks_for(h.n), kBlock, 0, h.stream>>>(cn, h.Dc.p, h.n);
}

void scale_problem(Handle &h) {
    hipStream_t s = h.stream;
    const int32_t m = h.m, n = h.n;
    k_fill<<<blocks_for(n), kBlock, 0, s>>>(h.Dc.p, 1.0, n);
    if (m > 0) k_fill<<<blocks_for(m), kBlock, 0, s>>>(h.Dr.p, 1.0, m);
    const int passes = h.opt.ruiz_iters + (h.opt.pock_chambolle ? 1 : 0);
    DBuf<double> rn, cn;
    rn.alloc(m);
    cn.alloc(n);
    const MatView VA = view(h.A), VT = view(h.AT);
    const int32_t nbA = h.A.nblocks(), nbT = h.AT.nblocks();
    if (h.dense) {
        dense_scale(h);
        transform_vectors(h);
        PDHG_HIP(hipStreamSynchronize(s));
        return;
    }
    for (int pass = 0; pass < passes && h.A.nnz > 0; ++pass) {
        const bool pc = pass >= h.opt.ruiz_iters;
        if (nbA) {
            if (pc) k_row_absnorm<false><<<nbA, kBlock, 0, s>>>(VA, rn.p);
            else k_row_absnorm<true><<<nbA, kBlock, 0, s>>>(VA, rn.p);
        }
        if (nbT) {
            if (pc) k_row_absnorm<false><<<nbT, kBlock, 0, s>>>(VT, cn.p);
            else k_row_absnorm<true><<<nbT, kBlock, 0, s>>>(VT, cn.p);
        }
        if (m > 0) k_factors<<<blocks_for(m), kBlock, 0, s>>>(rn.p, h.Dr.p, m);
        k_factors<<<blocks_for(n), kBlock, 0, s>>>(cn.p, h.Dc.p, n);
        if (nbA) k_scale_vals<<<nbA, kBlock, 0, s>>>(VA, rn.p, cn.p, 0);
        if (nbT) k_scale_vals<<<nbT, kBlock, 0, s>>>(VT, rn.p, cn.p, 1);
    }
    transform_vectors(h);
    PDHG_HIP(hipStreamSynchronize(s));
}

void transform_vectors(Handle &h) {
    const int32_t m = h.m, n = h.n;
    k_transform<<<blocks_for((int64_t)n + m), kBlock, 0, h.stream>>>(
        n, m, h.Dc.p, h.Dr.p, h.c_o.p, h.lv_o.p, h.uv_o.p, h.lc_o.p, h.uc_o.p, h.c.p, h.lv.p,
        h.uv.p, h.lc.p, h.uc.p);
}

// Largest eigenvalue of T = B'B for the Golub-Kahan bidiagonal B with
// diagonal alpha[0..k-1] and superdiagonal beta[0..k-2]: T_ii = alpha_i^2 +
// beta_{i-1}^2, T_i,i+1 = alpha_i beta_i. Bisection on the Sturm count over
// [0, Gershgorin bound] until the interval cannot be halved.
static int32_t sturm_count_below(const double *alpha, const double *beta, int32_t k, double x) {
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

double bidiag_lambda_max(const double *alpha, const double *beta, int32_t k) {
    double hi = 0.0;
    for (int32_t i = 0; i < k; ++i) {
        const double di = alpha[i] * alpha[i] + (i > 0 ? beta[i - 1] * beta[i - 1] : 0.0);
        const double el = i > 0 ? fabs(alpha[i - 1] * beta[i - 1]) : 0.0;
        const double er = i + 1 < k ? fabs(alpha[i] * beta[i]) : 0.0;
        hi = std::max(hi, di + el + er);
    }
    double lo = 0.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (sturm_count_below(alpha, beta, k, mid) == k)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

void estimate_steps(Handle &h) {
    hipStream_t s = h.stream;
    const int32_t m = h.m, n = h.n;
    h.norm_a = 0.0;
    h.power_iters = 0;
    if (h.A.nnz > 0 && m > 0) {
        // ||A~||_2 by Golub-Kahan-Lanczos bidiagonalisation from the start
        // vector: p = A~ v_k - beta_{k-1} u_{k-1}, alpha_k = |p|, u_k = p / alpha_k;
        // q = A~' u_k - alpha_k v_k, beta_k = |q|, v_{k+1} = q / beta_k. lam_k is
        // the largest eigenvalue of B_k'B_k; the host checks it every 16 steps.
        const int maxit = std::max(1, h.opt.power_max_iters);
        // workgroups of the products: the standard layout's blocks (CSR), the
        // dense passes' row and column blocks (dense)
        const int32_t nbA = h.dense ? h.nbm : h.A.nblocks(), nbT = h.dense ? h.nbn : h.AT.nblocks();
        const MatView VA = view(h.A), VT = view(h.AT);
        auto mul_a = [&](const double *vin, double *wout, double *part) {
            if (h.dense) dense_rows_sq(h, vin, wout, part);
            else k_spmv_sq<<<nbA, kBlock, 0, s>>>(VA, vin, wout, part);
        };
        auto mul_at = [&](const double *win, double *uout, double *part) {
            if (h.dense) dense_cols_sq(h, win, uout, part);
            else k_spmv_sq<<<nbT, kBlock, 0, s>>>(VT, win, uout, part);
        };
        const int32_t bm = (int32_t)blocks_for(m), bn = (int32_t)blocks_for(n);
        DBuf<double> v, w, u, z, pw, pu, ps, tot, hist;
        v.alloc(n);
        z.alloc(n);
        w.alloc(m);
        u.alloc(m);
        pw.alloc(std::max<int64_t>(nbA, 1));
        pu.alloc(std::max<int64_t>({(int64_t)nbT, (int64_t)bn, 1}));
        ps.alloc(std::max<int64_t>({(int64_t)bm, (int64_t)bn, 1}));
        tot.alloc(2);
        hist.alloc(2 * ((size_t)maxit + 2));
        PDHG_HIP(hipMemsetAsync(hist.p, 0, 2 * sizeof(double), s));
        PDHG_HIP(hipMemsetAsync(u.p, 0, (size_t)m * sizeof(double), s));
        k_power_start<<<bn, kBlock, 0, s>>>(h.perm_c.p, n, v.p, pu.p);
        k_total<1><<<1, kBlock, 0, s>>>(pu.p, bn, tot.p);
        k_div_sqrt<<<bn, kBlock, 0, s>>>(v.p, n, tot.p);
        const int batch = 16;
        std::vector<double> hh(2 * ((size_t)maxit + 2), 0.0);
        std::vector<double> al, be;
        double lam = 0.0, lam_prev = 0.0;
        int it_done = 0;
        bool stop = false;
        for (int it0 = 1; it0 <= maxit && !stop; it0 += batch) {
            const int it1 = std::min(maxit, it0 + batch - 1);
            for (int it = it0; it <= it1; ++it) {
                mul_a(v.p, w.p, pw.p);
                k_lanczos_sub<<<bm, kBlock, 0, s>>>(w.p, u.p, hist.p + 2 * (it - 1) + 1, m, ps.p);
                k_total<1><<<1, kBlock, 0, s>>>(ps.p, bm, tot.p);
                k_lanczos_scale<<<bm, kBlock, 0, s>>>(w.p, u.p, m, tot.p, hist.p + 2 * it);
                mul_at(u.p, z.p, pu.p);
                k_lanczos_sub<<<bn, kBlock, 0, s>>>(z.p, v.p, hist.p + 2 * it, n, ps.p);
                k_total<1><<<1, kBlock, 0, s>>>(ps.p, bn, tot.p + 1);
                k_lanczos_scale<<<bn, kBlock, 0, s>>>(z.p, v.p, n, tot.p + 1, hist.p + 2 * it + 1);
            }
            PDHG_HIP(hipMemcpyAsync(hh.data() + 2 * it0, hist.p + 2 * it0,
                                    sizeof(double) * 2 * (it1 - it0 + 1), hipMemcpyDeviceToHost,
                                    s));
            PDHG_HIP(hipStreamSynchronize(s));
            for (int it = it0; it <= it1; ++it) {
                const double a = hh[2 * it], b = hh[2 * it + 1];
                it_done = it;
                if (!(a > 0.0)) {
                    if (it == 1) lam = 0.0;
                    stop = true;
                    break;
                }
                al.push_back(a);
                be.push_back(b);
                lam = bidiag_lambda_max(al.data(), be.data(), it);
                if (!(b > 0.0)) {
                    stop = true;
                    break;
                }
                if (it > 1 && fabs(lam - lam_prev) <= h.opt.power_tol * lam) {
                    stop = true;
                    break;
                }
                lam_prev = lam;
            }
        }
        h.power_iters = it_done;
        h.norm_a = sqrt(lam);
    }
    h.eta = h.norm_a > 0.0 ? h.opt.step_safety / h.norm_a : 1.0;
}

void compute_weight(Handle &h) {
    hipStream_t s = h.stream;
    const int32_t m = h.m, n = h.n;
    const int nb = 64;
    DBuf<double> part, tot;
    part.alloc((size_t)nb * 4);
    tot.alloc(4);
    k_norm_sums<<<nb, kBlock, 0, s>>>(n, m, h.c.p, h.lc.p, h.uc.p, h.c_o.p, h.lc_o.p, h.uc_o.p,
                                       part.p);
    k_total<4><<<1, kBlock, 0, s>>>(part.p, nb, tot.p);
    double t[4];
    PDHG_HIP(hipMemcpyAsync(t, tot.p, sizeof(t), hipMemcpyDeviceToHost, s));
    PDHG_HIP(hipStreamSynchronize(s));
    const double cn = sqrt(t[0]), bn = sqrt(t[1]);
    h.omega0 = (cn > 1e-10 && bn > 1e-10) ? cn / bn : 1.0;
    h.cnorm = sqrt(t[2]);
    h.bnorm = sqrt(t[3]);
}


// LDS panels of the primal product (rows [0, R) of A~', scaled values) and the
// hot-column count of the dual product. The panel layout is built on the host
// from the rows kept at the matrix build and the scaled values of AT.
// f(t, lo, hi) on T host threads over contiguous ranges [lo, hi) of [0, n),
// T = min(16, hardware threads, n); the ranges are in order of t. An
// exception in any range is rethrown here after every thread has ended.
static int32_t host_threads(int64_t n) {
    const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>({16, hw, n}));
}
template <class F>
static void host_parallel(int64_t n, F f) {
    const int32_t T = host_threads(n);
    std::vector<std::exception_ptr> err((size_t)T);
    auto run = [&](int32_t t) {
        try {
            f(t, n * t / T, n * (t + 1) / T);
        } catch (...) {
            err[(size_t)t] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    for (int32_t t = 0; t + 1 < T; ++t) th.emplace_back(run, t);
    run(T - 1);
    for (auto &x : th) x.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

void build_fast_layouts(Handle &h) {
    hipStream_t s = h.stream;
    const int32_t m = h.m, n = h.n;
    int dev = 0, cus = 0;
    PDHG_HIP(hipGetDevice(&dev));
    PDHG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int32_t hot = h.opt.hot_cols < 0 ? (n > 262144 ? kHotMax : 0) : h.opt.hot_cols;
    h.hot_cols = (m > 0 && h.A.nslices > 0) ? std::min(hot, n) : 0;
    h.dual_wgs = 2 * std::max(1, cus);
    PanelMat &P = h.PT;
    if (P.R == 0) return;
    const int32_t R = P.R, S = P.S, RL = h.AT.R_long;
    const std::vector<int32_t> &rp = h.at_rowptr_host;
    const std::vector<int32_t> &ci = h.at_colidx_host;
    const int64_t nnz = rp[R];
    // scaled values of the covered rows: the CSR part of AT, then its first
    // sell_skip slices (entry k of row r at slice_ptr[s] + 64 k + lane)
    std::vector<int32_t> sptr((size_t)h.sell_skip + 1, 0);
    if (h.sell_skip > 0)
        PDHG_HIP(hipMemcpy(sptr.data(), h.AT.slice_ptr.p, sizeof(int32_t) * sptr.size(),
                           hipMemcpyDeviceToHost));
    const int64_t vend = h.sell_skip > 0 ? sptr[h.sell_skip] : rp[RL];
    std::vector<double> hv((size_t)vend);
    PDHG_HIP(hipMemcpy(hv.data(), h.AT.val.p, sizeof(double) * (size_t)vend, hipMemcpyDeviceToHost));
    auto value = [&](int32_t r, int64_t k) -> double {
        if (r < RL) return hv[(size_t)(rp[r] + k)];
        const int32_t q = r - RL;
        return hv[(size_t)sptr[q >> 6] + 64 * (size_t)k + (q & 63)];
    };
    P.vlen = m;
    P.P = (int32_t)ceil_div(m, S);
    P.W64 = (int32_t)ceil_div(P.P, 64);
    P.W = h.opt.panel_wgs < 0 ? kPanelWgsAuto : h.opt.panel_wgs;
    P.entries = nnz;
    // pieces (row, first entry, length) per panel, in row order
    struct Piece {
        int32_t row;
        int32_t len;
        int64_t e0;
        int32_t slot;
    };
    std::vector<std::vector<Piece>> pieces((size_t)P.P);
    std::vector<uint64_t> mask((size_t)P.W64 * R, 0);
    std::vector<int32_t> xcount((size_t)R, 0);
    int64_t nx = 0;
    {
        // rows in contiguous ranges per host thread, each collecting its pieces
        // per panel; the ranges are then joined in row order
        std::vector<std::vector<std::vector<Piece>>> local;
        std::vector<int64_t> lnx;
        const int32_t T = host_threads(R);
        local.resize((size_t)T, std::vector<std::vector<Piece>>((size_t)P.P));
        lnx.assign((size_t)T, 0);
        host_parallel(R, [&](int32_t t, int64_t r0, int64_t r1) {
            auto &mine = local[(size_t)t];
            for (int64_t r = r0; r < r1; ++r) {
                int64_t e = rp[(size_t)r];
                const int64_t e1 = rp[(size_t)r + 1];
                while (e < e1) {
                    const int32_t p = ci[(size_t)e] / S;   // entries of a row are sorted by y index
                    int64_t f = e;
                    while (f < e1 && ci[(size_t)f] / S == p) ++f;
                    mask[(size_t)(p >> 6) * R + (size_t)r] |= 1ull << (p & 63);
                    for (int64_t q = e; q < f; q += kPanelPiece) {
                        const int32_t len = (int32_t)std::min<int64_t>(kPanelPiece, f - q);
                        int32_t slot = -1;
                        if (q == e) {
                            slot = (int32_t)((int64_t)p * R + r);
                        } else {
                            slot = -2;   // numbered below, in row order
                            ++xcount[(size_t)r];
                            ++lnx[(size_t)t];
                        }
                        mine[(size_t)p].push_back(Piece{(int32_t)r, len, q, slot});
                    }
                    e = f;
                }
            }
        });
        for (int32_t t = 0; t < T; ++t) nx += lnx[(size_t)t];
        host_parallel(P.P, [&](int32_t, int64_t p0, int64_t p1) {
            for (int64_t p = p0; p < p1; ++p) {
                size_t total = 0;
                for (int32_t t = 0; t < T; ++t) total += local[(size_t)t][(size_t)p].size();
                std::vector<Piece> &v = pieces[(size_t)p];
                v.reserve(total);
                for (int32_t t = 0; t < T; ++t) {
                    std::vector<Piece> &l = local[(size_t)t][(size_t)p];
                    v.insert(v.end(), l.begin(), l.end());
                    std::vector<Piece>().swap(l);
                }
            }
        });
    }
    if ((int64_t)P.P * R + nx >= INT32_MAX) fail(PDHG_ERR_UNSUPPORTED, "too many panel partials");
    // extra pieces: slots P*R + x, x in row order then panel order
    std::vector<int32_t> xptr((size_t)R + 1, 0);
    for (int32_t r = 0; r < R; ++r) xptr[r + 1] = xptr[r] + xcount[(size_t)r];
    std::vector<int32_t> xslot((size_t)std::max<int64_t>(1, nx));
    std::vector<int32_t> xfill(xptr.begin(), xptr.end() - 1);
    for (int32_t p = 0; p < P.P; ++p)
        for (Piece &pc : pieces[(size_t)p])
            if (pc.slot == -2) {
                const int32_t x = xfill[(size_t)pc.row]++;
                pc.slot = (int32_t)((int64_t)P.P * R + x);
                xslot[(size_t)x] = pc.slot;
            }
    P.nx = (int32_t)nx;
    // SELL-64 slices per panel, pieces sorted by length (stable, longest
    // first). Per panel on host threads: the order by a counting sort on the
    // length (at most kPanelPiece), then, after the panels' sizes are added
    // up in panel order, each panel fills its own range of the arrays.
    std::vector<std::vector<int32_t>> order((size_t)P.P);
    std::vector<int64_t> p_entries((size_t)P.P, 0);
    std::vector<int32_t> p_slices((size_t)P.P, 0);
    host_parallel(P.P, [&](int32_t, int64_t p0, int64_t p1) {
        for (int64_t p = p0; p < p1; ++p) {
            const std::vector<Piece> &v = pieces[(size_t)p];
            std::vector<int32_t> cnt((size_t)kPanelPiece + 2, 0);
            for (const Piece &pc : v) ++cnt[(size_t)(kPanelPiece - pc.len + 1)];
            for (size_t b = 1; b < cnt.size(); ++b) cnt[b] += cnt[b - 1];
            std::vector<int32_t> &o = order[(size_t)p];
            o.resize(v.size());
            for (size_t q = 0; q < v.size(); ++q) o[(size_t)cnt[(size_t)(kPanelPiece - v[q].len)]++] = (int32_t)q;
            const int32_t ns = (int32_t)ceil_div((int64_t)v.size(), 64);
            int64_t ent = 0;
            for (int32_t sl = 0; sl < ns; ++sl) ent += (int64_t)64 * v[(size_t)o[(size_t)sl * 64]].len;
            p_entries[(size_t)p] = ent;
            p_slices[(size_t)p] = ns;
        }
    });
    std::vector<int32_t> pslice((size_t)P.P + 1, 0);
    std::vector<int64_t> ebase((size_t)P.P + 1, 0);
    for (int32_t p = 0; p < P.P; ++p) {
        pslice[(size_t)p + 1] = pslice[(size_t)p] + p_slices[(size_t)p];
        ebase[(size_t)p + 1] = ebase[(size_t)p] + p_entries[(size_t)p];
    }
    if (ebase[(size_t)P.P] >= (int64_t)INT32_MAX) fail(PDHG_ERR_UNSUPPORTED, "panel layout too large");
    std::vector<uint16_t> idx((size_t)ebase[(size_t)P.P], 0);
    std::vector<double> val((size_t)ebase[(size_t)P.P], 0.0);
    std::vector<int32_t> soff((size_t)pslice[(size_t)P.P] + 1, 0);
    std::vector<int32_t> slot((size_t)pslice[(size_t)P.P] * 64, -1);
    host_parallel(P.P, [&](int32_t, int64_t p0, int64_t p1) {
        for (int64_t p = p0; p < p1; ++p) {
            const std::vector<Piece> &v = pieces[(size_t)p];
            const std::vector<int32_t> &o = order[(size_t)p];
            const int32_t ns = p_slices[(size_t)p];
            size_t base = (size_t)ebase[(size_t)p];
            for (int32_t sl = 0; sl < ns; ++sl) {
                const size_t first = (size_t)sl * 64;
                const int32_t w = v[(size_t)o[first]].len;
                const size_t gs = (size_t)pslice[(size_t)p] + (size_t)sl;
                for (int32_t l = 0; l < 64; ++l) {
                    const size_t q = first + (size_t)l;
                    if (q >= v.size()) continue;
                    const Piece &pc = v[(size_t)o[q]];
                    slot[gs * 64 + (size_t)l] = pc.slot;
                    for (int32_t k = 0; k < pc.len; ++k) {
                        const int64_t e = pc.e0 + k;
                        idx[base + (size_t)64 * k + l] = (uint16_t)(ci[(size_t)e] - p * S);
                        val[base + (size_t)64 * k + l] = value(pc.row, e - rp[pc.row]);
                    }
                }
                base += (size_t)64 * w;
                soff[gs + 1] = (int32_t)base;
            }
        }
    });
    for (auto &v : pieces) std::vector<Piece>().swap(v);
    P.nslices = pslice[P.P];
    // workgroups: W per panel, all of a panel's workgroups on one XCD (workgroup
    // b runs on XCD b mod 8), so the panel's partial-sum lines meet in one L2
    std::vector<std::vector<std::pair<int32_t, int32_t>>> xcd(8);
    for (int32_t p = 0; p < P.P; ++p)
        for (int32_t g = 0; g < P.W; ++g) xcd[(size_t)(p % 8)].emplace_back(p, g);
    size_t longest = 0;
    for (const auto &l : xcd) longest = std::max(longest, l.size());
    std::vector<int32_t> wg_panel(8 * longest, -1), wg_rank(8 * longest, 0);
    for (int32_t x = 0; x < 8; ++x)
        for (size_t j = 0; j < xcd[(size_t)x].size(); ++j) {
            wg_panel[8 * j + (size_t)x] = xcd[(size_t)x][j].first;
            wg_rank[8 * j + (size_t)x] = xcd[(size_t)x][j].second;
        }
    P.nwg = (int32_t)wg_panel.size();
    auto upload = [&](auto &buf, const auto &v) {
        buf.alloc(v.size());
        PDHG_HIP(hipMemcpyAsync(buf.p, v.data(), sizeof(v[0]) * v.size(), hipMemcpyHostToDevice, s));
    };
    upload(P.idx, idx);
    upload(P.val, val);
    upload(P.soff, soff);
    upload(P.slot, slot);
    upload(P.pslice, pslice);
    upload(P.wg_panel, wg_panel);
    upload(P.wg_rank, wg_rank);
    upload(P.mask, mask);
    upload(P.xptr, xptr);
    upload(P.xslot, xslot);
    P.part.alloc((size_t)P.P * R + (size_t)nx);
    PDHG_HIP(hipStreamSynchronize(s));
    h.at_rowptr_host = {};
    h.at_colidx_host = {};
}
}  // namespace pdhg
