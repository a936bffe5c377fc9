// Internal declarations of libpdhg (not part of the public ABI).
//
// Layout in HBM: every vector is a contiguous FP64 array in the library's
// INTERNAL order. Rows of A and of A' (= columns of A) are permuted so that
// rows of similar length are adjacent (descending length class, stable inside
// a class); a segment table then gives each run of rows a fixed number of
// lanes per row. perm_r / perm_c map internal -> original indices.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "pdhg.h"

namespace pdhg {

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kMaxSeg = 40;      // length classes per matrix
constexpr int kShortMax = 64;    // rows up to this length go to SELL-64 slices

struct Error {
    pdhg_err code;
    std::string msg;
};

[[noreturn]] void fail(pdhg_err code, const std::string &msg);

// Device memory of the library's buffers. Blocks of 1 MiB and more are kept
// after release (up to 8 GiB per process, by device and exact size) and
// handed out again to an allocation of the same size: handles that are created
// and destroyed over and over (a batch per training step) then skip the
// driver's allocation and unmapping. device_free waits for the device first,
// as hipFree does, so no work in flight still uses a block that is reused.
// device_alloc returns nullptr when the device is out of memory (after giving
// the kept blocks back).
void *device_alloc(size_t bytes);
void device_free(void *p, size_t bytes);

#define PDHG_HIP(expr)                                                                  \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            ::pdhg::fail(PDHG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Owning device buffer.
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        const size_t bytes = (count ? count : 1) * sizeof(T);
        p = static_cast<T *>(device_alloc(bytes));
        if (!p) fail(PDHG_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        n = count;
    }
    void release() {
        if (p) device_free(p, (n ? n : 1) * sizeof(T));
        p = nullptr;
        n = 0;
    }
    T *get() const { return p; }
};

// A run of rows [row_begin, row_end) processed with 2^lanes_log2 lanes per
// row, starting at workgroup block_begin.
struct Seg {
    int32_t row_begin, row_end, lanes_log2, block_begin;
};
struct SegTable {
    Seg s[kMaxSeg];
    int32_t nseg;
    int32_t nblocks;
};

// Matrix in internal order, rows sorted by length (descending):
//  - rows [0, R_long) longer than the short-row limit: CSR (rowptr over these
//    rows, entries at the front of colidx/val), lane groups per the segment
//    table;
//  - rows [R_long, rows): SELL-64 slices. Slice s holds 64 consecutive rows;
//    entry k of lane l sits at slice_ptr[s] + 64 k + l for k < width(s),
//    width(s) = length of the slice's first (longest) row; shorter rows are
//    padded with (column 0, value 0.0). One thread per row.
struct HMat {
    int32_t rows = 0, cols = 0;
    int64_t nnz = 0;          // real entries
    int64_t stored = 0;       // entries incl. padding
    int32_t R_long = 0, nslices = 0;
    DBuf<int32_t> rowptr, colidx, slice_ptr;
    DBuf<double> val;
    SegTable seg{};
    int32_t nblocks() const { return seg.nblocks + (int32_t)((nslices + 3) / 4); }
};

// Kernel-argument view of an HMat.
struct MatView {
    const int32_t *rowptr;
    const int32_t *colidx;
    double *val;
    const int32_t *slice_ptr;
    int32_t rows, R_long, nslices, pad;
    SegTable seg;
};

inline MatView view(const HMat &M) {
    MatView v;
    v.rowptr = M.rowptr.p;
    v.colidx = M.colidx.p;
    v.val = M.val.p;
    v.slice_ptr = M.slice_ptr.p;
    v.rows = M.rows;
    v.R_long = M.R_long;
    v.nslices = M.nslices;
    v.pad = 0;
    v.seg = M.seg;
    return v;
}

// LDS panels for the product A~'y over rows [0, R) of A~' (the longest rows).
// The gathered vector y is cut into panels of S consecutive entries (S doubles
// fit in LDS). A sub-row is the part of a row whose entries fall in one panel;
// sub-rows longer than kPanelPiece are cut into pieces. Each panel stores its
// pieces as SELL-64 slices (pieces sorted by length, entries column-major in
// a slice, the y index relative to the panel in 16 bits), so one lane sums one
// piece in entry order. The first piece of sub-row (p, row) is stored to
// part[p * R + row] (bit p of the row's mask says the sub-row exists); further
// pieces go to part[P * R + x], listed per row in xptr / xslot.
constexpr int kPanelMax = 20480;   // doubles per LDS panel (160 KB, the most a workgroup may take)
constexpr int kPanelWgsAuto = 12;  // workgroups per panel of the automatic layout
constexpr int kHotMax = 20480;     // doubles of x_ext staged by the hot-column dual (160 KB)
constexpr int kPanelWaves = 16;    // waves per panel workgroup
constexpr int kPanelThreads = 64 * kPanelWaves;
constexpr int kPanelPiece = 128;   // longest piece one lane sums
struct PanelMat {
    int32_t R = 0, S = 0, P = 0, W64 = 0;   // rows, panel size, panels, mask words per row
    int32_t vlen = 0;                       // length of the gathered vector
    int32_t W = 0;                          // workgroups per panel
    int32_t nslices = 0, nwg = 0, nx = 0;
    int64_t entries = 0;                    // real entries
    DBuf<uint16_t> idx;      // soff[nslices] entries
    DBuf<double> val;
    DBuf<int32_t> soff;      // nslices + 1: first entry of each slice
    DBuf<int32_t> slot;      // nslices * 64: partial of each lane (-1: none)
    DBuf<int32_t> pslice;    // P + 1: first slice of each panel
    DBuf<int32_t> wg_panel;  // nwg: panel of each workgroup (-1: idle)
    DBuf<int32_t> wg_rank;   // nwg: rank of the workgroup within its panel
    DBuf<uint64_t> mask;     // [W64][R]
    DBuf<int32_t> xptr;      // R + 1
    DBuf<int32_t> xslot;     // nx
    DBuf<double> part;       // P * R + nx
};

struct PanelView {
    const uint16_t *idx;
    const double *val;
    const int32_t *soff, *slot, *pslice, *wg_panel, *wg_rank;
    const uint64_t *mask;
    const int32_t *xptr, *xslot;
    double *part;
    int32_t R, S, P, W64, vlen, W;
};

inline PanelView view(const PanelMat &M) {
    PanelView v;
    v.idx = M.idx.p;
    v.val = M.val.p;
    v.soff = M.soff.p;
    v.slot = M.slot.p;
    v.pslice = M.pslice.p;
    v.wg_panel = M.wg_panel.p;
    v.wg_rank = M.wg_rank.p;
    v.mask = M.mask.p;
    v.xptr = M.xptr.p;
    v.xslot = M.xslot.p;
    v.part = M.part.p;
    v.R = M.R;
    v.S = M.S;
    v.P = M.P;
    v.W64 = M.W64;
    v.vlen = M.vlen;
    v.W = M.W;
    return v;
}

// Solver scalars kept on the device; the controller kernel owns them.
struct DevState {
    double tau, sigma, omega, eta;
    double r_start, r_prev;
    double kkt, rel_p, rel_d, rel_g, pobj, dobj, abs_p, abs_d, abs_g;
    double last_r;
    int64_t t_next;      // iteration index of the next check
    int64_t k_base;      // inner counter of the first plain iteration after a check
    int64_t k_check;     // inner counter at the last check
    int64_t plain_prev;  // plain iterations after the last check
    int64_t restarts;
    int64_t t_done;      // iteration index at which the solve stopped
    int32_t done, status, action, first;
    double ray_scale;      // 1 / |objective| of the certifying ray
    int32_t anchor_valid;  // products of the restart anchor are stored
    int32_t pad;
};

// Constants the controller needs.
struct CtlConst {
    double eps, bnorm, cnorm, eta;
    double beta_suff, beta_nec, beta_art;
    double norm_q;
    int32_t qp;
    int32_t detect;        // 1: infeasibility tests (LP)
    double eps_pinf, eps_dinf;
    int32_t term;          // stop on: 0 the KKT error, 1 the primal residual, 2 the dual residual
    int32_t pad;
};

struct Handle {
    int32_t m = 0, n = 0;
    pdhg_options opt{};
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr;
    HMat A, AT;
    DBuf<int32_t> perm_r, perm_c;        // internal -> original
    DBuf<double> Dr, Dc;                 // scaling, internal order
    DBuf<double> c, lc, uc, lv, uv;      // scaled data
    DBuf<double> c_o, lc_o, uc_o, lv_o, uv_o;  // original data, internal order
    DBuf<double> x, y, x0, y0, xhat, yhat, xext, aty;
    DBuf<double> pn, pm;                 // per-workgroup partial sums of a check
    DBuf<double> prn, prm;               // per-workgroup ray sums / maxima of a check
    DBuf<double> p0, q0, phat, qhat;     // A~x0, A~'y0 of the anchor; A~xhat, A~'yhat
    DBuf<double> qv0, qvhat;             // QP: Q~x0 of the anchor; Q~xbar of this check
    DBuf<double> scratch;                // reductions of setup / power iteration
    DBuf<DevState> st;
    DevState *st_host = nullptr;         // pinned ring of status copies
    int st_ring = 4;
    double eta = 1.0, omega0 = 1.0, norm_a = 0.0, norm_q = 0.0;
    double cnorm = 0.0, bnorm = 0.0;
    int32_t power_iters = 0;
    double setup_seconds = 0.0;
    int32_t polish = 0;                  // 0 solve; 1 / 2 primal / dual polishing phase
    hipGraphExec_t chunk_exec = nullptr;
    hipGraph_t chunk_graph = nullptr;
    // quadratic term Q~ = D_c Q D_c (rAPDHG), internal order
    int32_t q_kind = 0;                  // 0 none, PDHG_FMT_CSR, PDHG_FMT_DENSE, PDHG_FMT_LOWRANK_DIAG
    int32_t q_rank = 0;
    DBuf<int32_t> q_rp, q_ci;            // CSR
    DBuf<double> q_va, q_dense, q_f, q_d;  // CSR values, dense n x n, factor n x r, diagonal
    DBuf<double> xbar, ybar, qv_in, qv, qpart, qt;
    // dense constraint matrix (row-major, scaled in place) and column-pass partials
    bool dense = false;
    DBuf<double> Ad, dpart;
    int32_t nbn = 0, nbm = 0;            // workgroups of the column / row check passes
    // iteration layouts of a large sparse A~ (the check iterations use them for
    // their products with A~' as well; those with A~ run on A):
    // LDS panels for the long rows of A~' (their products run beside the SELL-64
    // rest of A~' on stream2), and the leading x_ext entries staged in LDS by
    // the dual product
    PanelMat PT;
    int32_t sell_skip = 0;               // SELL-64 slices of AT that the panels cover
    int32_t hot_cols = 0;                // 0: the dual product gathers x_ext from memory
    int32_t dual_wgs = 0;                // persistent workgroups of the hot dual product
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<int32_t> at_rowptr_host; // rows of A~' the panels may cover (kept from the build)
    std::vector<int32_t> at_colidx_host;
    ~Handle();
};

// ---- loss heads (heads.hip) ---------------------------------------------
void head_linear_costs(hipStream_t s, int32_t B, int32_t n, int32_t p, const double *f,
                       const double *W, double *c);
void head_regret(hipStream_t s, int32_t B, int32_t n, const double *ct, const double *x,
                 const double *vs, double *loss);
void head_linear_costs_backward(hipStream_t s, int32_t B, int32_t n, int32_t p, const double *f,
                                const double *gc, double *gW);
void head_linear_costs_backward_noalloc(hipStream_t s, int32_t B, int32_t n, int32_t p,
                                        const double *f, const double *gc, double *gW);
void head_qp_value(hipStream_t s, int32_t B, int32_t n, int32_t r, const double *F,
                   const double *d, const double *c, const double *x, double *value, double *gx);
void head_spo_costs(hipStream_t s, int32_t B, int32_t n, const double *c_hat, const double *c_true,
                    double *out);
void head_spo_plus(hipStream_t s, int32_t B, int32_t n, const double *c_hat, const double *c_true,
                   const double *w_star, const double *z_star, const double *w_tilde, double *loss,
                   double *grad);
void head_pfy_costs(hipStream_t s, int32_t B, int32_t M, int32_t n, const double *c_hat,
                    const double *Z, double eps, double *out);
void head_pfy(hipStream_t s, int32_t B, int32_t M, int32_t n, const double *c_hat,
              const double *w_star, const double *Z, double eps, const double *w_samples, double *loss,
              double *grad);

// ---- setup (setup.hip) ---------------------------------------------------
void build_matrices(Handle &h, const pdhg_problem &p);
void validate_and_load_vectors(Handle &h, const pdhg_problem &p);
void scale_problem(Handle &h);
void transform_vectors(Handle &h);
void estimate_steps(Handle &h);
void compute_weight(Handle &h);
void build_fast_layouts(Handle &h);
SegTable make_segments(const std::vector<int32_t> &class_count, int32_t rows);
void validate_csr(hipStream_t s, const int32_t *rowptr, const int32_t *colidx, const double *val,
                  int32_t m, int32_t n, int64_t nnz);
void validate_vectors(hipStream_t s, int32_t n, int32_t m, const double *c, const double *lv,
                      const double *uv, const double *lc, const double *uc);
void plain_transpose(hipStream_t s, int32_t rows, int32_t cols, int64_t nnz, const int32_t *rowptr,
                     const int32_t *colidx, const double *val, int32_t *rowptr_t,
                     int32_t *colidx_t, double *val_t);
void check_flag(hipStream_t s, const int32_t *dflag, const char *what);
void permute_csr(hipStream_t s, int32_t rows, int32_t cols, int64_t nnz, const int32_t *rowptr,
                 const int32_t *colidx, const double *val, const int32_t *perm_r,
                 const int32_t *perm_c, int32_t *out_rp, int32_t *out_ci, double *out_va);
double now_seconds();
void order_after_stream(hipStream_t own, hipEvent_t ev, void *caller);
void check_options(const pdhg_options &o);

// ---- dense matrices (dense_kernels.hip) --------------------------------------
void dense_build(Handle &h, const pdhg_problem &p);
void dense_scale(Handle &h);
void dense_primal(Handle &h, int32_t j);
void dense_dual(Handle &h, int32_t j);
void dense_primal_check(Handle &h, double tau_override);
void dense_dual_check(Handle &h, double sigma_override);
void dense_check_sums(Handle &h);
void dense_rows_sq(Handle &h, const double *v, double *out, double *partials);
void dense_cols_sq(Handle &h, const double *w, double *out, double *partials);
int32_t dense_row_blocks(const Handle &h);
int32_t check_n_blocks(const Handle &h);
int32_t dense_col_blocks(const Handle &h);
void launch_factors(Handle &h, double *rn, double *cn);

// ---- rAPDHG (qp_kernels.hip) -------------------------------------------------
void qp_build(Handle &h, const pdhg_problem &p);
void qp_estimate_norm(Handle &h);
void launch_qp_iteration(Handle &h, int32_t j);
void launch_qp_check(Handle &h, int32_t chunk_plain, int32_t is_last, int32_t last_status);
void launch_qp_finalize(Handle &h, double *x_out, double *y_out);
void launch_qp_init(Handle &h);
void launch_qp_debug_step(Handle &h, int64_t k, double omega);

// ---- batched solver (batch.hip) ---------------------------------------------
struct BatchHandle;
BatchHandle *batch_create(const pdhg_batch_problem &p, const pdhg_options &o, void *stream);
void batch_solve(BatchHandle &b, const double *x_init, const double *y_init, double *x_out,
                 double *y_out, pdhg_result *res);
void batch_set_launch(BatchHandle &b, int32_t threads, int32_t workgroups);
int32_t batch_autotune(BatchHandle &b, int32_t iterations);
void batch_unrolled_forward(BatchHandle &b, int64_t T, int32_t replay, double *x_out, double *y_out);
void batch_backward(BatchHandle &b, const double *gx, const double *gy, double *gc, double *glc,
                    double *guc, double *gd);
void batch_update_data(BatchHandle &b, const double *c, const double *lc, const double *uc,
                       const double *lv, const double *uv);
void batch_destroy(BatchHandle *b);

// ---- iteration kernels (lp_kernels.hip) -------------------------------------
void launch_primal(Handle &h, int32_t j, hipEvent_t *timing = nullptr);
void launch_dual(Handle &h, int32_t j);
void launch_primal_check(Handle &h, double tau_override = -1.0);
void launch_dual_check(Handle &h, double sigma_override = -1.0);
void launch_check_sums(Handle &h);
void launch_controller(Handle &h, int32_t chunk_plain, int32_t is_last, int32_t last_status);
void launch_apply(Handle &h);
void launch_make_ray(Handle &h, int32_t status);
void launch_zero_finite(Handle &h, double *v, int32_t len);
void launch_init_point(Handle &h, const double *x_init, const double *y_init);
void launch_finalize(Handle &h, double *x_out, double *y_out);
void launch_reset_state(Handle &h);
void launch_set_step(Handle &h, double tau, double sigma, int64_t k);
void launch_debug_halpern(Handle &h, int64_t k, double *xnew_int, double *ynew_int);
void launch_gather(hipStream_t s, const int32_t *perm, const double *src, double *dst, int32_t len);
void launch_scatter(hipStream_t s, const int32_t *perm, const double *src, double *dst, int32_t len);
void launch_scatter_scaled(hipStream_t s, const int32_t *perm, const double *scale,
                           const double *src, double *dst, int32_t len);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace pdhg
