// C ABI of libpdhg and the host loop that runs the device-resident solve.
//
// The solve runs in check periods of check_every iterations: one check
// iteration (PDHG point kept, KKT and fixed-point residual, controller,
// restart-or-Halpern) followed by check_every - 1 plain iterations (two fused
// kernels each). A period is replayed as one HIP graph. Every kernel of a
// period returns at once when the controller has set the done flag, so the
// host can keep two periods in flight and poll a pinned status copy without
// stalling the GPU.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <deque>
#include <new>
#include <unordered_map>
#include <mutex>
#include <map>

#include "batch_internal.hpp"
#include "common.hpp"

namespace pdhg {

static thread_local std::string g_err = "";
constexpr int kTimingEvents = 7;   // per timed plain iteration

void fail(pdhg_err code, const std::string &msg) { throw Error{code, msg}; }

namespace {
constexpr size_t kKeepMinBytes = size_t(1) << 20;
constexpr size_t kKeepMaxBytes = size_t(8) << 30;
struct BlockCache {
    std::mutex mu;
    std::multimap<std::pair<int, size_t>, void *> free;   // (device, bytes) -> block
    std::unordered_map<void *, int> device;                // device of every large block
    size_t kept = 0;
};
// never destroyed: blocks still kept at exit go back with the process
BlockCache &block_cache() {
    static BlockCache *c = new BlockCache;
    return *c;
}
// hipFree every kept block of device `dev` (the current device)
void release_kept(BlockCache &c, int dev) {
    for (auto it = c.free.begin(); it != c.free.end();) {
        if (it->first.first == dev) {
            (void)hipFree(it->second);
            c.device.erase(it->second);
            c.kept -= it->first.second;
            it = c.free.erase(it);
        } else {
            ++it;
        }
    }
}
}  // namespace

void *device_alloc(size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    BlockCache &c = block_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    if (bytes >= kKeepMinBytes) {
        auto it = c.free.find({dev, bytes});
        if (it != c.free.end()) {
            void *p = it->second;
            c.free.erase(it);
            c.kept -= bytes;
            return p;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        release_kept(c, dev);
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    if (bytes >= kKeepMinBytes) c.device[p] = dev;
    return p;
}

void device_free(void *p, size_t bytes) {
    if (!p) return;
    BlockCache &c = block_cache();
    if (bytes >= kKeepMinBytes) {
        int dev = -1, cur = 0;
        {
            std::lock_guard<std::mutex> lock(c.mu);
            auto d = c.device.find(p);
            if (d != c.device.end()) dev = d->second;
        }
        if (dev >= 0 && hipGetDevice(&cur) == hipSuccess) {
            // work in flight may still use the block: wait for its device
            if (cur != dev) (void)hipSetDevice(dev);
            const bool idle = hipDeviceSynchronize() == hipSuccess;
            if (cur != dev) (void)hipSetDevice(cur);
            std::lock_guard<std::mutex> lock(c.mu);
            if (idle && c.kept + bytes <= kKeepMaxBytes) {
                c.free.insert({{dev, bytes}, p});
                c.kept += bytes;
                return;
            }
            c.device.erase(p);
        }
    }
    (void)hipFree(p);
}

Handle::~Handle() {
    if (chunk_exec) (void)hipGraphExecDestroy(chunk_exec);
    if (chunk_graph) (void)hipGraphDestroy(chunk_graph);
    if (st_host) (void)hipHostFree(st_host);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (stream2) (void)hipStreamDestroy(stream2);
    if (stream) (void)hipStreamDestroy(stream);
}

template <class F>
static pdhg_err guarded(F &&f) {
    try {
        f();
        return PDHG_OK;
    } catch (const Error &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return PDHG_ERR_OOM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return PDHG_ERR_HIP;
    } catch (...) {
        g_err = "unknown failure";
        return PDHG_ERR_HIP;
    }
}

double now_seconds() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}
static double now_s() { return now_seconds(); }

// Make `own` wait for the work already queued on the caller's stream.
void order_after_stream(hipStream_t own, hipEvent_t ev, void *caller) {
    PDHG_HIP(hipEventRecord(ev, reinterpret_cast<hipStream_t>(caller)));
    PDHG_HIP(hipStreamWaitEvent(own, ev, 0));
}
static void order_after(Handle &h, void *caller) { order_after_stream(h.stream, h.ev_in, caller); }

void check_options(const pdhg_options &o) {
    if (!(o.eps > 0.0) || o.iteration_limit < 1 || o.check_every < 1 || o.ruiz_iters < 0 ||
        !(o.gamma >= 0.0 && o.gamma <= 1.0) || !(o.step_safety > 0.0 && o.step_safety <= 1.0) ||
        o.power_max_iters < 1 || !(o.power_tol >= 0.0) || o.display_frequency < 1 ||
        o.panel_rows < -1 || o.panel_rows > kPanelMax || o.panel_min_len < -1 ||
        o.panel_wgs < -1 || o.panel_wgs == 0 || o.panel_wgs > 64 || o.hot_cols < -1 ||
        o.hot_cols > kHotMax)
        fail(PDHG_ERR_INVALID_ARG, "option out of range");
}

static void enqueue_check(Handle &h, int32_t chunk_plain, int32_t is_last, int32_t last_status) {
    if (h.q_kind) {
        launch_qp_check(h, chunk_plain, is_last, last_status);
        return;
    }
    launch_primal_check(h);
    launch_dual_check(h);
    launch_check_sums(h);
    launch_controller(h, chunk_plain, is_last, last_status);
    launch_apply(h);
}

static void enqueue_plain(Handle &h, int32_t j) {
    if (h.q_kind) {
        launch_qp_iteration(h, j);
        return;
    }
    launch_primal(h, j);
    launch_dual(h, j);
}

static void build_graph(Handle &h) {
    if (h.chunk_exec) return;
    const int32_t C = h.opt.check_every;
    PDHG_HIP(hipStreamBeginCapture(h.stream, hipStreamCaptureModeThreadLocal));
    enqueue_check(h, C - 1, 0, 0);
    for (int32_t j = 1; j < C; ++j) enqueue_plain(h, j);
    hipGraph_t g = nullptr;
    PDHG_HIP(hipStreamEndCapture(h.stream, &g));
    h.chunk_graph = g;
    PDHG_HIP(hipGraphInstantiate(&h.chunk_exec, g, nullptr, nullptr, 0));
}

static void print_check(const DevState &s) {
    fprintf(stderr,
            "pdhg t=%-8lld restarts=%-4lld omega=%.3e kkt=%.3e (p %.2e d %.2e g %.2e) obj=%.10e "
            "r=%.17e r_start=%.17e r_prev=%.17e\n",
            (long long)s.t_done, (long long)s.restarts, s.omega, s.kkt, s.rel_p, s.rel_d,
            s.rel_g, s.pobj, s.last_r, s.r_start, s.r_prev);
}

static void run_solve(Handle &h, const double *x_init, const double *y_init, double *x_out,
                      double *y_out, pdhg_result *res) {
    const double t0 = now_s();
    hipStream_t s = h.stream;
    launch_reset_state(h);
    launch_init_point(h, x_init, y_init);
    if (h.q_kind) launch_qp_init(h);
    const int32_t C = h.opt.check_every;
    const int64_t L = h.opt.iteration_limit;
    // graphs hold the solve's controller constants: polishing phases run unrolled
    const bool graphs = h.opt.use_graph && !h.polish;
    if (graphs) build_graph(h);

    std::vector<hipEvent_t> tev;
    int64_t timing_t = -1;
    int timing_slot = -1;
    std::vector<hipEvent_t> ring(h.st_ring);
    for (auto &e : ring) PDHG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    std::deque<int> inflight;
    int64_t t = 0, chunk = 0;
    bool stop = false;
    int64_t checks_seen = 0;
    DevState timing_state{};
    bool have_timing_state = false;
    try {
        while (!stop && t < L) {
            bool final = false;
            const bool time_up = h.opt.time_limit_s > 0.0 && now_s() - t0 > h.opt.time_limit_s;
            int64_t plain = 0;
            if (time_up) {
                enqueue_check(h, 0, 1, PDHG_TIME_LIMIT);
                final = true;
            } else if (t == L - 1) {
                enqueue_check(h, 0, 1, PDHG_ITERATION_LIMIT);
                final = true;
            } else {
                plain = std::min<int64_t>(C - 1, L - 2 - t);
                const bool timed = h.opt.timing_chunk >= 0 && chunk == h.opt.timing_chunk &&
                                   plain == C - 1 && tev.empty() && !h.q_kind;
                if (plain == C - 1 && graphs && !timed) {
                    PDHG_HIP(hipGraphLaunch(h.chunk_exec, s));
                } else {
                    enqueue_check(h, (int32_t)plain, 0, 0);
                    if (timed) {
                        tev.resize(kTimingEvents * (size_t)plain);
                        for (auto &e : tev) PDHG_HIP(hipEventCreate(&e));
                        timing_t = t;
                    }
                    for (int32_t j = 1; j <= plain; ++j) {
                        if (!timed) {
                            enqueue_plain(h, j);
                            continue;
                        }
                        // events: reference, the primal step's kernels on each stream
                        // (start / end pairs), then around the dual step
                        hipEvent_t *e = &tev[kTimingEvents * (size_t)(j - 1)];
                        PDHG_HIP(hipEventRecord(e[0], s));
                        launch_primal(h, j, e + 1);
                        PDHG_HIP(hipEventRecord(e[5], s));
                        launch_dual(h, j);
                        PDHG_HIP(hipEventRecord(e[6], s));
                    }
                }
            }
            const int slot = (int)(chunk % h.st_ring);
            PDHG_HIP(hipMemcpyAsync(&h.st_host[slot], h.st.p, sizeof(DevState),
                                    hipMemcpyDeviceToHost, s));
            PDHG_HIP(hipEventRecord(ring[slot], s));
            if (timing_t == t && timing_slot < 0) timing_slot = slot;
            inflight.push_back(slot);
            t += 1 + plain;
            ++chunk;
            const size_t depth = final ? 0 : 2;
            while (inflight.size() > depth) {
                const int q = inflight.front();
                inflight.pop_front();
                PDHG_HIP(hipEventSynchronize(ring[q]));
                const DevState &sv = h.st_host[q];
                if (q == timing_slot) {
                    timing_state = sv;
                    have_timing_state = true;
                    timing_slot = -2;
                }
                ++checks_seen;
                if (h.opt.verbose && (checks_seen % h.opt.display_frequency) == 0) print_check(sv);
                if (sv.done) stop = true;
            }
            if (final) stop = true;
        }
        PDHG_HIP(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipStreamSynchronize(s);
        for (auto &e : ring) (void)hipEventDestroy(e);
        for (auto &e : tev) (void)hipEventDestroy(e);
        throw;
    }
    DevState fin;
    PDHG_HIP(hipMemcpy(&fin, h.st.p, sizeof(DevState), hipMemcpyDeviceToHost));
    if (fin.done && (fin.status == PDHG_PRIMAL_INFEASIBLE || fin.status == PDHG_DUAL_INFEASIBLE))
        launch_make_ray(h, fin.status);
    if (h.q_kind)
        launch_qp_finalize(h, x_out, y_out);
    else
        launch_finalize(h, x_out, y_out);
    PDHG_HIP(hipStreamSynchronize(s));
    if (h.opt.verbose) print_check(fin);
    double kp = 0.0, kd = 0.0;
    int32_t samples = 0;
    // the timed period counts only if the solve was still running after its check
    if (!tev.empty() && have_timing_state && !timing_state.done) {
        // primal step: earliest start to latest end of its kernels on the two
        // streams (times from the reference event); dual step: its own events
        for (size_t j = 0; j + kTimingEvents - 1 < tev.size(); j += kTimingEvents) {
            float t1 = 0.f, t2 = 0.f, t3 = 0.f, t4 = 0.f, d = 0.f;
            PDHG_HIP(hipEventElapsedTime(&t1, tev[j], tev[j + 1]));
            PDHG_HIP(hipEventElapsedTime(&t2, tev[j], tev[j + 2]));
            PDHG_HIP(hipEventElapsedTime(&t3, tev[j], tev[j + 3]));
            PDHG_HIP(hipEventElapsedTime(&t4, tev[j], tev[j + 4]));
            PDHG_HIP(hipEventElapsedTime(&d, tev[j + 5], tev[j + 6]));
            kp += std::max(t2, t4) - std::min(t1, t3);
            kd += d;
            ++samples;
        }
    }
    for (auto &e : ring) (void)hipEventDestroy(e);
    for (auto &e : tev) (void)hipEventDestroy(e);
    if (res) {
        memset(res, 0, sizeof(*res));
        res->status = fin.done ? fin.status : PDHG_ITERATION_LIMIT;
        res->iterations = fin.t_done + 1;
        res->restarts = fin.restarts;
        res->primal_obj = fin.pobj;
        res->dual_obj = fin.dobj;
        res->rel_primal_res = fin.rel_p;
        res->rel_dual_res = fin.rel_d;
        res->rel_gap = fin.rel_g;
        res->kkt_rel = fin.kkt;
        res->solve_seconds = now_s() - t0;
        res->setup_seconds = h.setup_seconds;
        res->eta = h.eta;
        res->omega = fin.omega;
        res->norm_a = h.norm_a;
        res->norm_q = h.norm_q;
        res->power_iters = h.power_iters;
        res->kernel_samples = samples;
        res->kernel_primal_ms = samples ? kp / samples : 0.0;
        res->kernel_dual_ms = samples ? kd / samples : 0.0;
    }
}

}  // namespace pdhg

using namespace pdhg;

// The caller's stream given at create: every call first waits for the work
// already queued there (its inputs may have been produced by it).
struct pdhg_handle {
    Handle h;
    void *caller = nullptr;
};

extern "C" {

void pdhg_options_default(pdhg_options *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->eps = 1e-4;
    o->iteration_limit = INT64_MAX;
    o->time_limit_s = 0.0;
    o->check_every = 64;
    o->ruiz_iters = 10;
    o->pock_chambolle = 1;
    o->gamma = 1.0;
    o->step_safety = 0.998;
    o->restart_sufficient = 0.2;
    o->restart_necessary = 0.8;
    o->restart_artificial = 0.36;
    o->power_tol = 1e-7;
    o->power_max_iters = 2000;
    o->verbose = 0;
    o->display_frequency = 10;
    o->use_graph = 1;
    o->timing_chunk = -1;
    o->eps_primal_infeasible = 1e-8;
    o->eps_dual_infeasible = 1e-8;
    o->feasibility_polishing = 0;
    o->eps_feas_polish = 1e-6;
    o->panel_rows = -1;
    o->panel_min_len = -1;
    o->panel_wgs = -1;
    o->hot_cols = -1;
}

const char *pdhg_last_error(void) { return g_err.c_str(); }

int32_t pdhg_version(void) { return 100; }

pdhg_err pdhg_create(const pdhg_problem *prob, const pdhg_options *opt, void *stream,
                     pdhg_handle **out) {
    if (out) *out = nullptr;
    pdhg_handle *ph = nullptr;
    pdhg_err rc = guarded([&] {
        if (!prob || !out) fail(PDHG_ERR_INVALID_ARG, "NULL problem or output pointer");
        const pdhg_problem &p = *prob;
        if (p.m < 0 || p.n < 1) fail(PDHG_ERR_INVALID_ARG, "need m >= 0 and n >= 1");
        if (p.mem != PDHG_MEM_HOST && p.mem != PDHG_MEM_DEVICE)
            fail(PDHG_ERR_INVALID_ARG, "mem must be PDHG_MEM_HOST or PDHG_MEM_DEVICE");
        if (p.a_format != PDHG_FMT_CSR && p.a_format != PDHG_FMT_DENSE)
            fail(PDHG_ERR_INVALID_ARG, "a_format must be PDHG_FMT_CSR or PDHG_FMT_DENSE");
        if (p.a_format == PDHG_FMT_DENSE && p.q_format != PDHG_FMT_NONE)
            fail(PDHG_ERR_UNSUPPORTED, "quadratic objectives need a CSR constraint matrix");
        if (p.a_format == PDHG_FMT_DENSE && p.m > 0 && !p.a_dense)
            fail(PDHG_ERR_INVALID_ARG, "NULL dense matrix");
        if (p.q_format != PDHG_FMT_NONE && p.q_format != PDHG_FMT_CSR &&
            p.q_format != PDHG_FMT_DENSE && p.q_format != PDHG_FMT_LOWRANK_DIAG)
            fail(PDHG_ERR_INVALID_ARG, "unknown q_format");
        if (p.a_format == PDHG_FMT_CSR &&
            (!p.a_rowptr || (p.a_nnz > 0 && (!p.a_colidx || !p.a_val)) || p.a_nnz < 0 ||
             p.a_nnz >= INT32_MAX))
            fail(PDHG_ERR_INVALID_ARG, "bad CSR arrays or nnz");
        if (!p.c || !p.lv || !p.uv || (p.m > 0 && (!p.lc || !p.uc)))
            fail(PDHG_ERR_INVALID_ARG, "NULL objective or bound vector");
        pdhg_options o;
        if (opt)
            o = *opt;
        else
            pdhg_options_default(&o);
        check_options(o);
        const double t0 = now_s();
        ph = new pdhg_handle();
        Handle &h = ph->h;
        h.m = p.m;
        h.n = p.n;
        h.opt = o;
        PDHG_HIP(hipStreamCreateWithFlags(&h.stream, hipStreamNonBlocking));
        PDHG_HIP(hipEventCreateWithFlags(&h.ev_in, hipEventDisableTiming));
        ph->caller = stream;
        order_after(h, stream);
        h.st.alloc(1);
        h.dense = p.a_format == PDHG_FMT_DENSE;
        if (h.dense) {
            dense_build(h, p);
            h.nbn = dense_col_blocks(h);
            h.nbm = h.m > 0 ? dense_row_blocks(h) : 0;
        } else {
            build_matrices(h, p);
            h.nbn = h.AT.nblocks();
            h.nbm = h.A.nblocks();
        }
        validate_and_load_vectors(h, p);
        scale_problem(h);
        estimate_steps(h);
        compute_weight(h);
        if (p.q_format != PDHG_FMT_NONE) {
            qp_build(h, p);
            qp_estimate_norm(h);
        } else if (!h.dense) {
            build_fast_layouts(h);
            h.nbn = check_n_blocks(h);
            if (h.PT.R > 0) {
                PDHG_HIP(hipStreamCreateWithFlags(&h.stream2, hipStreamNonBlocking));
                PDHG_HIP(hipEventCreateWithFlags(&h.ev_fork, hipEventDisableTiming));
                PDHG_HIP(hipEventCreateWithFlags(&h.ev_join, hipEventDisableTiming));
            }
        }
        h.pn.alloc((size_t)std::max(1, h.nbn) * 6);
        h.pm.alloc((size_t)std::max(1, h.nbm) * 4);
        // the checks also test infeasibility rays
        h.prn.alloc((size_t)std::max(1, h.nbn) * 4);
        h.prm.alloc((size_t)std::max(1, h.nbm) * 3);
        h.q0.alloc((size_t)h.n);
        h.qhat.alloc((size_t)h.n);
        h.p0.alloc((size_t)std::max(1, h.m));
        h.phat.alloc((size_t)std::max(1, h.m));
        if (h.q_kind) {
            h.qv0.alloc((size_t)h.n);
            h.qvhat.alloc((size_t)h.n);
        }
        PDHG_HIP(hipHostMalloc(reinterpret_cast<void **>(&h.st_host),
                               sizeof(DevState) * h.st_ring, hipHostMallocDefault));
        memset(h.st_host, 0, sizeof(DevState) * h.st_ring);
        PDHG_HIP(hipStreamSynchronize(h.stream));
        h.setup_seconds = now_s() - t0;
        *out = ph;
    });
    if (rc != PDHG_OK) delete ph;
    return rc;
}

// Feasibility polishing of an optimal LP point (x_out, y_out; original space,
// device): the primal phase solves the LP with c = 0 from x, the dual phase
// the LP with its finite bounds set to 0 from y, each to its own residual
// <= eps_feas_polish; the handle's data is restored after. res receives the
// KKT terms of the polished point for the original LP.
static void polish(Handle &h, double *x_out, double *y_out, pdhg_result *res) {
    hipStream_t s = h.stream;
    const int32_t m = h.m, n = h.n;
    const size_t bn = sizeof(double) * n, bm = sizeof(double) * m;
    DBuf<double> sc, slc, suc, slv, suv, xs, ys, xt, yt;
    for (auto *b : {&sc, &slv, &suv, &xs, &xt}) b->alloc(n);
    for (auto *b : {&slc, &suc, &ys, &yt}) b->alloc(std::max(1, m));
    PDHG_HIP(hipMemcpyAsync(sc.p, h.c_o.p, bn, hipMemcpyDeviceToDevice, s));
    PDHG_HIP(hipMemcpyAsync(slv.p, h.lv_o.p, bn, hipMemcpyDeviceToDevice, s));
    PDHG_HIP(hipMemcpyAsync(suv.p, h.uv_o.p, bn, hipMemcpyDeviceToDevice, s));
    PDHG_HIP(hipMemcpyAsync(xs.p, x_out, bn, hipMemcpyDeviceToDevice, s));
    if (m > 0) {
        PDHG_HIP(hipMemcpyAsync(slc.p, h.lc_o.p, bm, hipMemcpyDeviceToDevice, s));
        PDHG_HIP(hipMemcpyAsync(suc.p, h.uc_o.p, bm, hipMemcpyDeviceToDevice, s));
        PDHG_HIP(hipMemcpyAsync(ys.p, y_out, bm, hipMemcpyDeviceToDevice, s));
    }
    auto restore = [&] {
        h.polish = 0;
        PDHG_HIP(hipMemcpyAsync(h.c_o.p, sc.p, bn, hipMemcpyDeviceToDevice, s));
        PDHG_HIP(hipMemcpyAsync(h.lv_o.p, slv.p, bn, hipMemcpyDeviceToDevice, s));
        PDHG_HIP(hipMemcpyAsync(h.uv_o.p, suv.p, bn, hipMemcpyDeviceToDevice, s));
        if (m > 0) {
            PDHG_HIP(hipMemcpyAsync(h.lc_o.p, slc.p, bm, hipMemcpyDeviceToDevice, s));
            PDHG_HIP(hipMemcpyAsync(h.uc_o.p, suc.p, bm, hipMemcpyDeviceToDevice, s));
        }
        transform_vectors(h);
        compute_weight(h);
    };
    pdhg_result r1, r2;
    try {
        // primal phase: c = 0
        PDHG_HIP(hipMemsetAsync(h.c_o.p, 0, bn, s));
        transform_vectors(h);
        compute_weight(h);
        h.polish = 1;
        run_solve(h, xs.p, nullptr, x_out, yt.p, &r1);
        // dual phase: c restored, finite bounds 0
        PDHG_HIP(hipMemcpyAsync(h.c_o.p, sc.p, bn, hipMemcpyDeviceToDevice, s));
        launch_zero_finite(h, h.lv_o.p, n);
        launch_zero_finite(h, h.uv_o.p, n);
        launch_zero_finite(h, h.lc_o.p, m);
        launch_zero_finite(h, h.uc_o.p, m);
        transform_vectors(h);
        compute_weight(h);
        h.polish = 2;
        run_solve(h, nullptr, m > 0 ? ys.p : nullptr, xt.p, y_out, &r2);
    } catch (...) {
        try {
            restore();
        } catch (...) {
        }
        throw;
    }
    // the original data back, and the KKT terms of (x_out, y_out) from one check
    restore();
    launch_reset_state(h);
    launch_init_point(h, x_out, m > 0 ? y_out : nullptr);
    PDHG_HIP(hipMemcpyAsync(h.xhat.p, h.x.p, bn, hipMemcpyDeviceToDevice, s));
    if (m > 0) PDHG_HIP(hipMemcpyAsync(h.yhat.p, h.y.p, bm, hipMemcpyDeviceToDevice, s));
    launch_check_sums(h);
    launch_controller(h, 0, 1, PDHG_OPTIMAL);
    DevState ev;
    PDHG_HIP(hipMemcpyAsync(&ev, h.st.p, sizeof(DevState), hipMemcpyDeviceToHost, s));
    PDHG_HIP(hipStreamSynchronize(s));
    res->iterations += r1.iterations + r2.iterations;
    res->polish_iterations = r1.iterations + r2.iterations;
    res->primal_obj = ev.pobj;
    res->dual_obj = ev.dobj;
    res->rel_primal_res = ev.rel_p;
    res->rel_dual_res = ev.rel_d;
    res->rel_gap = ev.rel_g;
    res->kkt_rel = ev.kkt;
    res->solve_seconds += r1.solve_seconds + r2.solve_seconds;
}

pdhg_err pdhg_solve(pdhg_handle *ph, const double *x_init, const double *y_init, double *x_out,
                    double *y_out, pdhg_result *res) {
    return guarded([&] {
        if (!ph || !x_out || (ph->h.m > 0 && !y_out))
            fail(PDHG_ERR_INVALID_ARG, "NULL handle or output pointer");
        Handle &h = ph->h;
        order_after(h, ph->caller);
        pdhg_result local;
        pdhg_result *r = res ? res : &local;
        run_solve(h, x_init, y_init, x_out, y_out, r);
        if (h.opt.feasibility_polishing && !h.q_kind && r->status == PDHG_OPTIMAL)
            polish(h, x_out, y_out, r);
    });
}

pdhg_err pdhg_update_data(pdhg_handle *ph, const double *c, const double *lc, const double *uc,
                          const double *lv, const double *uv) {
    return guarded([&] {
        if (!ph) fail(PDHG_ERR_INVALID_ARG, "NULL handle");
        Handle &h = ph->h;
        order_after(h, ph->caller);
        hipStream_t s = h.stream;
        DBuf<double> tc, tl, tu, tlv, tuv;
        // validate the new data in original order before taking it
        pdhg_problem p;
        memset(&p, 0, sizeof(p));
        p.m = h.m;
        p.n = h.n;
        p.mem = PDHG_MEM_DEVICE;
        tc.alloc(h.n);
        tlv.alloc(h.n);
        tuv.alloc(h.n);
        tl.alloc(h.m);
        tu.alloc(h.m);
        launch_scatter(s, h.perm_c.p, h.c_o.p, tc.p, h.n);
        launch_scatter(s, h.perm_c.p, h.lv_o.p, tlv.p, h.n);
        launch_scatter(s, h.perm_c.p, h.uv_o.p, tuv.p, h.n);
        launch_scatter(s, h.perm_r.p, h.lc_o.p, tl.p, h.m);
        launch_scatter(s, h.perm_r.p, h.uc_o.p, tu.p, h.m);
        p.c = c ? c : tc.p;
        p.lv = lv ? lv : tlv.p;
        p.uv = uv ? uv : tuv.p;
        p.lc = lc ? lc : tl.p;
        p.uc = uc ? uc : tu.p;
        validate_and_load_vectors(h, p);
        // D_r, D_c and A~ are kept; only the transformed vectors change.
        transform_vectors(h);
        compute_weight(h);
        PDHG_HIP(hipStreamSynchronize(s));
    });
}

pdhg_err pdhg_debug_step(pdhg_handle *ph, const double *x, const double *y, const double *x0,
                         const double *y0, int64_t k, double tau, double sigma, double *xhat,
                         double *yhat, double *xnew, double *ynew) {
    return guarded([&] {
        if (!ph || !x || !x0 || (ph->h.m > 0 && (!y || !y0)))
            fail(PDHG_ERR_INVALID_ARG, "NULL handle or state pointer");
        if (!(tau > 0.0) || !(sigma > 0.0) || k < 0)
            fail(PDHG_ERR_INVALID_ARG, "tau, sigma must be > 0 and k >= 0");
        Handle &h = ph->h;
        order_after(h, ph->caller);
        if (h.q_kind) fail(PDHG_ERR_UNSUPPORTED, "pdhg_debug_step is for LP handles");
        hipStream_t s = h.stream;
        launch_reset_state(h);
        launch_gather(s, h.perm_c.p, x, h.x.p, h.n);
        launch_gather(s, h.perm_c.p, x0, h.x0.p, h.n);
        launch_gather(s, h.perm_r.p, y, h.y.p, h.m);
        launch_gather(s, h.perm_r.p, y0, h.y0.p, h.m);
        launch_primal_check(h, tau);
        launch_dual_check(h, sigma);
        DBuf<double> xn, yn;
        xn.alloc(h.n);
        yn.alloc(h.m);
        launch_debug_halpern(h, k, xn.p, yn.p);
        if (xhat) launch_scatter(s, h.perm_c.p, h.xhat.p, xhat, h.n);
        if (yhat) launch_scatter(s, h.perm_r.p, h.yhat.p, yhat, h.m);
        if (xnew) launch_scatter(s, h.perm_c.p, xn.p, xnew, h.n);
        if (ynew) launch_scatter(s, h.perm_r.p, yn.p, ynew, h.m);
        PDHG_HIP(hipStreamSynchronize(s));
    });
}

pdhg_err pdhg_debug_plain_step(pdhg_handle *ph, const double *x, const double *y,
                               const double *x0, const double *y0, int64_t k, double tau,
                               double sigma, double *xnew, double *ynew) {
    return guarded([&] {
        if (!ph || !x || !x0 || (ph->h.m > 0 && (!y || !y0)))
            fail(PDHG_ERR_INVALID_ARG, "NULL handle or state pointer");
        if (!(tau > 0.0) || !(sigma > 0.0) || k < 0)
            fail(PDHG_ERR_INVALID_ARG, "tau, sigma must be > 0 and k >= 0");
        Handle &h = ph->h;
        order_after(h, ph->caller);
        if (h.q_kind) fail(PDHG_ERR_UNSUPPORTED, "pdhg_debug_plain_step is for LP handles");
        hipStream_t s = h.stream;
        launch_reset_state(h);
        launch_set_step(h, tau, sigma, k);
        launch_gather(s, h.perm_c.p, x, h.x.p, h.n);
        launch_gather(s, h.perm_c.p, x0, h.x0.p, h.n);
        launch_gather(s, h.perm_r.p, y, h.y.p, h.m);
        launch_gather(s, h.perm_r.p, y0, h.y0.p, h.m);
        launch_primal(h, 1);
        launch_dual(h, 1);
        if (xnew) launch_scatter(s, h.perm_c.p, h.x.p, xnew, h.n);
        if (ynew) launch_scatter(s, h.perm_r.p, h.y.p, ynew, h.m);
        PDHG_HIP(hipStreamSynchronize(s));
    });
}

pdhg_err pdhg_debug_qp_step(pdhg_handle *ph, const double *x, const double *y,
                            const double *xbar, const double *ybar, int64_t k, double omega,
                            double *xn, double *yn, double *xbarn, double *ybarn) {
    return guarded([&] {
        if (!ph || !x || !xbar || (ph->h.m > 0 && (!y || !ybar)))
            fail(PDHG_ERR_INVALID_ARG, "NULL handle or state pointer");
        if (!(omega > 0.0) || k < 0) fail(PDHG_ERR_INVALID_ARG, "omega must be > 0 and k >= 0");
        Handle &h = ph->h;
        order_after(h, ph->caller);
        if (!h.q_kind) fail(PDHG_ERR_UNSUPPORTED, "pdhg_debug_qp_step is for QP handles");
        hipStream_t s = h.stream;
        launch_gather(s, h.perm_c.p, x, h.x.p, h.n);
        launch_gather(s, h.perm_c.p, xbar, h.xbar.p, h.n);
        launch_gather(s, h.perm_r.p, y, h.y.p, h.m);
        launch_gather(s, h.perm_r.p, ybar, h.ybar.p, h.m);
        launch_qp_debug_step(h, k, omega);
        if (xn) launch_scatter(s, h.perm_c.p, h.x.p, xn, h.n);
        if (yn) launch_scatter(s, h.perm_r.p, h.y.p, yn, h.m);
        if (xbarn) launch_scatter(s, h.perm_c.p, h.xbar.p, xbarn, h.n);
        if (ybarn) launch_scatter(s, h.perm_r.p, h.ybar.p, ybarn, h.m);
        PDHG_HIP(hipStreamSynchronize(s));
    });
}

pdhg_err pdhg_get_scaling(pdhg_handle *ph, double *dr, double *dc, double *scalars,
                          int32_t *power_iters) {
    return guarded([&] {
        if (!ph) fail(PDHG_ERR_INVALID_ARG, "NULL handle");
        Handle &h = ph->h;
        order_after(h, ph->caller);
        if (dr) launch_scatter(h.stream, h.perm_r.p, h.Dr.p, dr, h.m);
        if (dc) launch_scatter(h.stream, h.perm_c.p, h.Dc.p, dc, h.n);
        PDHG_HIP(hipStreamSynchronize(h.stream));
        if (scalars) {
            scalars[0] = h.eta;
            scalars[1] = h.omega0;
            scalars[2] = h.norm_a;
            scalars[3] = h.norm_q;
        }
        if (power_iters) *power_iters = h.power_iters;
    });
}

void pdhg_destroy(pdhg_handle *ph) {
    if (!ph) return;
    (void)hipStreamSynchronize(ph->h.stream);
    delete ph;
}

struct pdhg_batch {
    BatchHandle *b;
    void *caller;   // as for pdhg_handle
};

static void order_after_caller(pdhg_batch *pb) { order_after_stream(pb->b->stream, pb->b->ev, pb->caller); }

pdhg_err pdhg_batch_create(const pdhg_batch_problem *prob, const pdhg_options *opt, void *stream,
                           pdhg_batch **out) {
    if (out) *out = nullptr;
    return guarded([&] {
        if (!prob || !out) fail(PDHG_ERR_INVALID_ARG, "NULL problem or output pointer");
        pdhg_options o;
        if (opt)
            o = *opt;
        else
            pdhg_options_default(&o);
        check_options(o);
        BatchHandle *b = batch_create(*prob, o, stream);
        *out = new pdhg_batch{b, stream};
    });
}

pdhg_err pdhg_batch_solve(pdhg_batch *pb, const double *x_init, const double *y_init,
                          double *x_out, double *y_out, pdhg_result *res) {
    return guarded([&] {
        if (!pb || !x_out || !y_out) fail(PDHG_ERR_INVALID_ARG, "NULL batch or output pointer");
        order_after_caller(pb);
        batch_solve(*pb->b, x_init, y_init, x_out, y_out, res);
    });
}

pdhg_err pdhg_batch_set_launch(pdhg_batch *pb, int32_t threads, int32_t workgroups) {
    return guarded([&] {
        if (!pb) fail(PDHG_ERR_INVALID_ARG, "NULL batch");
        batch_set_launch(*pb->b, threads, workgroups);
    });
}

pdhg_err pdhg_batch_autotune(pdhg_batch *pb, int32_t iterations, int32_t *best_threads) {
    return guarded([&] {
        if (!pb || iterations < 1) fail(PDHG_ERR_INVALID_ARG, "NULL batch or iterations < 1");
        order_after_caller(pb);
        const int32_t t = batch_autotune(*pb->b, iterations);
        if (best_threads) *best_threads = t;
    });
}

pdhg_err pdhg_batch_update_data(pdhg_batch *pb, const double *c, const double *lc,
                                const double *uc, const double *lv, const double *uv) {
    return guarded([&] {
        if (!pb) fail(PDHG_ERR_INVALID_ARG, "NULL batch");
        order_after_caller(pb);
        batch_update_data(*pb->b, c, lc, uc, lv, uv);
    });
}

pdhg_err pdhg_batch_unrolled_forward(pdhg_batch *pb, int64_t T, int32_t replay, double *x_out,
                                     double *y_out) {
    return guarded([&] {
        if (!pb || !x_out || !y_out) fail(PDHG_ERR_INVALID_ARG, "NULL batch or output pointer");
        order_after_caller(pb);
        batch_unrolled_forward(*pb->b, T, replay, x_out, y_out);
    });
}

pdhg_err pdhg_batch_unrolled_backward(pdhg_batch *pb, const double *gx, const double *gy,
                                      double *gc, double *glc, double *guc, double *gd) {
    return guarded([&] {
        if (!pb || !gx || !gc) fail(PDHG_ERR_INVALID_ARG, "NULL batch, gx or gc");
        order_after_caller(pb);
        batch_backward(*pb->b, gx, gy, gc, glc, guc, gd);
    });
}

void pdhg_batch_destroy(pdhg_batch *pb) {
    if (!pb) return;
    batch_destroy(pb->b);
    delete pb;
}

}  // extern "C"

// ---- loss heads --------------------------------------------------------------

pdhg_err pdhg_linear_costs(int32_t B, int32_t n, int32_t p, const double *f, const double *W,
                           double *c_hat, void *stream) {
    return guarded([&] {
        if (B < 0 || n < 0 || p < 1 || p > 64) fail(PDHG_ERR_INVALID_ARG, "need B, n >= 0, 1 <= p <= 64");
        if ((int64_t)B * n > 0 && (!f || !W || !c_hat)) fail(PDHG_ERR_INVALID_ARG, "NULL array");
        head_linear_costs(reinterpret_cast<hipStream_t>(stream), B, n, p, f, W, c_hat);
    });
}

pdhg_err pdhg_regret(int32_t B, int32_t n, const double *c_true, const double *x,
                     const double *v_star, double *loss, void *stream) {
    return guarded([&] {
        if (B < 0 || n < 0) fail(PDHG_ERR_INVALID_ARG, "need B, n >= 0");
        if (B > 0 && (!c_true || !x || !v_star || !loss)) fail(PDHG_ERR_INVALID_ARG, "NULL array");
        head_regret(reinterpret_cast<hipStream_t>(stream), B, n, c_true, x, v_star, loss);
    });
}

pdhg_err pdhg_linear_costs_backward(int32_t B, int32_t n, int32_t p, const double *f,
                                    const double *gc, double *gW, void *stream) {
    return guarded([&] {
        if (B < 0 || n < 0 || p < 1 || p > 64) fail(PDHG_ERR_INVALID_ARG, "need B, n >= 0, 1 <= p <= 64");
        if (!gW || ((int64_t)B * n > 0 && (!f || !gc))) fail(PDHG_ERR_INVALID_ARG, "NULL array");
        head_linear_costs_backward(reinterpret_cast<hipStream_t>(stream), B, n, p, f, gc, gW);
    });
}

pdhg_err pdhg_linear_costs_backward_noalloc(int32_t B, int32_t n, int32_t p, const double *f,
                                            const double *gc, double *gW, void *stream) {
    return guarded([&] {
        if (B < 0 || n < 0 || p < 1 || p > 64) fail(PDHG_ERR_INVALID_ARG, "need B, n >= 0, 1 <= p <= 64");
        if (!gW || ((int64_t)B * n > 0 && (!f || !gc))) fail(PDHG_ERR_INVALID_ARG, "NULL array");
        head_linear_costs_backward_noalloc(reinterpret_cast<hipStream_t>(stream), B, n, p, f, gc, gW);
    });
}

pdhg_err pdhg_qp_value(int32_t B, int32_t n, int32_t r, const double *F, const double *d,
                       const double *c, const double *x, double *value, double *gx, void *stream) {
    return guarded([&] {
        if (B < 0 || n < 0 || r < 0 || r > 32) fail(PDHG_ERR_INVALID_ARG, "need B, n >= 0, 0 <= r <= 32");
        if (B > 0 && (!d || !c || !x || !value || (r > 0 && !F)))
            fail(PDHG_ERR_INVALID_ARG, "NULL array");
        head_qp_value(reinterpret_cast<hipStream_t>(stream), B, n, r, F, d, c, x, value, gx);
    });
}

pdhg_err pdhg_spo_plus_costs(int32_t B, int32_t n, const double *c_hat, const double *c_true,
                             double *c_out, void *stream) {
    return guarded([&] {
        if (B < 0 || n < 0) fail(PDHG_ERR_INVALID_ARG, "need B, n >= 0");
        if ((int64_t)B * n > 0 && (!c_hat || !c_true || !c_out)) fail(PDHG_ERR_INVALID_ARG, "NULL array");
        head_spo_costs(reinterpret_cast<hipStream_t>(stream), B, n, c_hat, c_true, c_out);
    });
}

pdhg_err pdhg_spo_plus(int32_t B, int32_t n, const double *c_hat, const double *c_true,
                       const double *w_star, const double *z_star, const double *w_tilde, double *loss,
                       double *grad, void *stream) {
    return guarded([&] {
        if (B < 0 || n < 0) fail(PDHG_ERR_INVALID_ARG, "need B, n >= 0");
        if (B > 0 && (!z_star || !loss || (n > 0 && (!c_hat || !c_true || !w_star || !w_tilde || !grad))))
            fail(PDHG_ERR_INVALID_ARG, "NULL array");
        head_spo_plus(reinterpret_cast<hipStream_t>(stream), B, n, c_hat, c_true, w_star, z_star, w_tilde,
                      loss, grad);
    });
}

pdhg_err pdhg_pfy_costs(int32_t B, int32_t M, int32_t n, const double *c_hat, const double *Z, double eps,
                        double *c_out, void *stream) {
    return guarded([&] {
        if (B < 0 || M < 1 || n < 0) fail(PDHG_ERR_INVALID_ARG, "need B, n >= 0, M >= 1");
        if (!std::isfinite(eps)) fail(PDHG_ERR_INVALID_ARG, "eps must be finite");
        if ((int64_t)B * n > 0 && (!c_hat || !Z || !c_out)) fail(PDHG_ERR_INVALID_ARG, "NULL array");
        head_pfy_costs(reinterpret_cast<hipStream_t>(stream), B, M, n, c_hat, Z, eps, c_out);
    });
}

pdhg_err pdhg_pfy(int32_t B, int32_t M, int32_t n, const double *c_hat, const double *w_star,
                  const double *Z, double eps, const double *w_samples, double *loss, double *grad,
                  void *stream) {
    return guarded([&] {
        if (B < 0 || M < 1 || n < 0) fail(PDHG_ERR_INVALID_ARG, "need B, n >= 0, M >= 1");
        if (!std::isfinite(eps)) fail(PDHG_ERR_INVALID_ARG, "eps must be finite");
        if (B > 0 && (!loss || (n > 0 && (!c_hat || !w_star || !Z || !w_samples || !grad))))
            fail(PDHG_ERR_INVALID_ARG, "NULL array");
        head_pfy(reinterpret_cast<hipStream_t>(stream), B, M, n, c_hat, w_star, Z, eps, w_samples, loss,
                 grad);
    });
}
