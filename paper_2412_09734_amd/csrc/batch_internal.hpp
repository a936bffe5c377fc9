// Host-side state of a batch (shared by batch.hip and batch_qp.hip).
#pragma once

#include <vector>

#include "common.hpp"

namespace pdhg {

struct BatchRes {
    double pobj, dobj, rel_p, rel_d, rel_g, kkt, omega, eta;
    int64_t iterations, restarts;
    int32_t status, power_iters;
};

struct BatchHandle {
    int32_t B = 0, shared = 0, m = 0, n = 0;   // shared: per-instance m, n; ragged: totals
    int64_t nnz = 0;
    int32_t vec_m = 0, vec_n = 0;              // lengths of the row / column vectors
    pdhg_options opt{};
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    DBuf<int32_t> row_off, col_off, arp, aci, trp, tci, power_iters, queue;
    DBuf<double> ava, tva, Dr, Dc, eta;
    DBuf<double> c_o, lc_o, uc_o, lv_o, uv_o, c, lc, uc, lv, uv;
    DBuf<double> x, x0, xh, xe, aty, y, y0, yh;
    DBuf<BatchRes> res;
    int32_t threads = 256;
    bool threads_set = false;            // chosen by set_launch / autotune
    int32_t workgroups = 0;
    double setup_seconds = 0.0;
    const double *x_init_ = nullptr, *y_init_ = nullptr;
    double *x_out_ = nullptr, *y_out_ = nullptr;
    std::vector<int32_t> row_off_h, col_off_h;
    // SELL-64 copies of the scaled A~ and A~' (built after scaling): slices
    // never cross instances; slice s of instance b is sfirst[b] + local row / 64
    DBuf<int32_t> asp, asci, asfirst, tsp, tsci, tsfirst;
    DBuf<double> asva, tsva;
    DBuf<double> lhist;                   // Lanczos coefficients during setup
    DBuf<double> rp0, rq0, rph, rqh;      // LP: A~x0, A~'y0 of each anchor; this check's products
    // QP batches: Q_b = F F' + diag(d_b), F shared (scaled copy), d per instance
    int32_t q_rank = 0;
    double q_eta = 1.0;                   // step size of the shared A~ (host copy)
    int32_t q_cus = 0;                    // compute units of the device
    DBuf<double> qF, qd_o, qdd, normq, xbar, ybar, qv_, qres;
    DBuf<double> ckpt, vseg, bxb, byb, bw, bqv;
    DBuf<double> vall;                    // QP: every momentum point of the unrolled forward
    bool u_vall = false;
    // unrolled iterations: schedule, masks and reverse-pass scratch
    int64_t unrolled_T = 0;
    int32_t nmax = 0, mmax = 0;           // largest instance (LDS sizing)
    int32_t onchip = 1;                   // use the on-chip solve when it fits
    int32_t resident = 1;                 // keep narrow shared matrices in registers
    int32_t as_wmax = 0, ts_wmax = 0;     // widest SELL-64 slice of A~ and A~
    DBuf<uint8_t> u_restart;
    DBuf<double> u_omega, u_ba;
    DBuf<int32_t> u_kk;
    DBuf<uint64_t> u_xmask, u_ymask;
    DBuf<int64_t> u_xoff, u_yoff;
    ~BatchHandle() {
        if (ev) (void)hipEventDestroy(ev);
        if (stream) (void)hipStreamDestroy(stream);
    }
};


// QP batches (batch_qp.hip)
void bqp_create(BatchHandle &h, const pdhg_batch_problem &p);
void bqp_solve(BatchHandle &h, const double *x_init, const double *y_init, double *x_out,
               double *y_out, pdhg_result *res);
void bqp_unrolled(BatchHandle &h, int64_t T, int32_t replay, double *x_out, double *y_out);
void bqp_backward(BatchHandle &h, const double *gx, const double *gy, double *gc, double *glc,
                  double *guc, double *gd);

}  // namespace pdhg
