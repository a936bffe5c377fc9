"""Benchmark: plain r2HPDHG on the large sparse LP (m=1e6, n=2e6, Zipf column
degrees, rows scaled by LogUniform(1e-2, 1e2)), FP64, relative KKT <= 1e-4.

One step = the whole hot path on one LP whose data is already in HBM:
pdhg_create (layout, Ruiz + Pock-Chambolle scaling, power iteration) +
pdhg_solve to the tolerance + pdhg_destroy. value = LPs solved per second.

Prints one JSON line with a roofline object for the dominant iteration kernel
(HIP-event durations measured inside the timed solves) and the CPU oracle's
rate on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LPs solved/sec @1e-4 rel KKT (batched vs plain); PDHG iter HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(m: int, n: int, nnz: int) -> dict:
    """Algorithmic HBM bytes of one launch of each plain-iteration kernel.

    primal (rows of A'): A' values + column indices (12 B per entry) and row
    pointers; reads x, x0, c, l_v, u_v; writes x_ext, x; gathers y once.
    dual (rows of A): A values + indices and row pointers; reads y, y0, l_c,
    u_c; writes y; gathers x_ext once."""
    primal = 12 * nnz + 4 * (n + 1) + 8 * (5 * n + 2 * n) + 8 * m
    dual = 12 * nnz + 4 * (m + 1) + 8 * (4 * m + 1 * m) + 8 * n
    return {"primal": primal, "dual": dual}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sparse_zipf_1Mx2M_pmc_traffic.txt")
KERNEL_SOURCES = ["lp_kernels.hip", "device.hpp", "common.hpp", "setup.hip"]


def measured_traffic(step: str):
    """HBM bytes per iteration step ('primal' or 'dual': the sum over the step's
    kernels) from the committed FETCH_SIZE / WRITE_SIZE counter summary
    (calibrated against a 1 GiB copy), or None when the kernel sources changed
    since the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2412_09734_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("kernel-sources-sha256:", "traffic-bytes ")))
    if fields.get("kernel-sources-sha256", "").strip() != h.hexdigest():
        return None
    v = fields.get(f"traffic-bytes {step}")
    return int(v) if v else None


def stream_peak() -> dict:
    """Achievable HBM bandwidth on this GPU: the best of 5 timed 1 GiB
    device-to-device copies (2 GiB moved each), of 5 triads a = b + 2c on
    1 GiB vectors (3 GiB moved each) and of 5 sums of a 1 GiB vector (a read
    stream, as the solver's passes mostly are), in GB/s."""
    import torch
    n = 1 << 27
    b = torch.ones(n, dtype=torch.float64, device="cuda:0")
    c = torch.ones(n, dtype=torch.float64, device="cuda:0")
    a = torch.empty_like(b)
    out = {}
    for name, op, moved in (("copy", lambda: a.copy_(b), 2 * 8 * n),
                            ("triad", lambda: torch.add(b, c, alpha=2.0, out=a), 3 * 8 * n),
                            ("read", lambda: torch.sum(b), 8 * n)):
        op()
        best = float("inf")
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            op()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        out[name] = round(moved / best / 1e9, 1)
    del a, b, c
    torch.cuda.empty_cache()
    return out


def cpu_baseline(lp, gpu_iters: int, gpu_power_iters: int) -> dict:
    """The oracle on a bounded sample of the same LP: its scaling, then 40
    iterations (checks at the first and last), timed on all host threads the
    box gives the process (OMP_NUM_THREADS, else every core: the products run
    on them) and on one; the per-LP time is extrapolated to the GPU's
    power-iteration and iteration counts (each power step costs about one
    iteration's two products)."""
    import oracle
    oracle.build(force=False)
    sample_iters = 40
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)

    def run(t):
        oracle.set_threads(t)
        t0 = time.perf_counter()
        orc = oracle.Oracle(lp, power_max_iters=1, iteration_limit=sample_iters)
        t_setup = time.perf_counter() - t0
        t1 = time.perf_counter()
        orc.solve()
        t_iter = (time.perf_counter() - t1) / sample_iters
        orc.close()
        return t_setup, t_iter, t_setup + (gpu_power_iters + gpu_iters) * t_iter

    s_all, i_all, lp_all = run(threads)
    s_one, i_one, lp_one = run(1)
    oracle.set_threads(1)
    return {"value": 1.0 / lp_all, "unit": "LPs/s", "cores": threads, "kind": "oracle",
            "single_core_value": 1.0 / lp_one,
            "sample": (f"oracle scaling + {sample_iters} iterations on the full LP, extrapolated to "
                       f"{gpu_power_iters} power steps + {gpu_iters} iterations per LP: on {threads} "
                       f"threads (products parallel, the rest serial) scaling {s_all:.2f} s and "
                       f"{i_all * 1e3:.1f} ms per iteration; on 1 thread {s_one:.2f} s and "
                       f"{i_one * 1e3:.1f} ms")}


def batched_vs_plain(loop_sample: int = 8, steps: int = 3) -> dict:
    """The batched half of the metric in the default run: 2,048 grid min-cost
    flow LPs sharing one incidence matrix, created (layout, scaling, step
    size) and solved in one persistent launch, against the plain solver looped
    over the first instances (create + solve each), in LPs solved per second."""
    import numpy as np
    import torch

    import gen
    from paper_2412_09734_amd.solver import BatchSolver, Solver

    dev = torch.device("cuda:0")
    B = 2048
    sb = gen.grid_mincost_batch(batch=B, seed=gen.seed_for(3, 0))
    kw = {k: (torch.from_numpy(np.ascontiguousarray(v)).to(dev, torch.int32 if v.dtype.kind in "iu"
                                                             else torch.float64)
              if isinstance(v, np.ndarray) else v)
          for k, v in dict(shared_a=True, batch=B, m=sb.m, n=sb.n, rowptr=sb.rowptr, colidx=sb.colidx,
                           val=sb.val, c=sb.c, lc=sb.lc, uc=sb.uc, lv=sb.lv, uv=sb.uv).items()}
    with BatchSolver(**kw) as bs:
        best = bs.autotune(128)
        bs.set_launch(best)
        bs.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved = 0
    for _ in range(steps):
        with BatchSolver(**kw) as bs:
            bs.set_launch(best)
            _, _, res = bs.solve()
            solved += sum(r["status"] == 1 for r in res)
    torch.cuda.synchronize()
    batch_rate = solved / (time.perf_counter() - t0)
    inst = [sb.instance(b) for b in range(loop_sample)]
    with Solver.from_lp(inst[0]) as s:
        s.solve()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ok = 0
    for lp in inst:
        with Solver.from_lp(lp) as s:
            _, _, r = s.solve()
        ok += r["status"] == 1
    torch.cuda.synchronize()
    loop_rate = ok / (time.perf_counter() - t1)
    return {"workload": f"{B} min-cost-flow LPs sharing a 32x32 grid incidence (1024 x 3968), KKT <= 1e-4",
            "batched_lps_per_s": round(batch_rate, 2), "plain_looped_lps_per_s": round(loop_rate, 2),
            "speedup": round(batch_rate / loop_rate, 1), "threads_per_instance": int(best),
            "batched_steps": steps, "looped_instances": loop_sample}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=1_000_000)
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other", action="store_true",
                    help="sparse workload: skip the portfolio-QP and dense-knapsack figures of the default run "
                         "(also skipped with --iteration-limit or --layout)")
    ap.add_argument("--no-batched", action="store_true",
                    help="sparse workload: skip the batched-vs-plain grid measurement")
    ap.add_argument("--iteration-limit", type=int, default=0,
                    help="stop every solve after this many iterations (profiling runs only)")
    ap.add_argument("--eps", type=float, default=1e-4,
                    help="sparse workloads: relative KKT tolerance of the solve (default 1e-4)")
    ap.add_argument("--no-infeasibility-tests", action="store_true",
                    help="batched and SPO+ workloads: switch the infeasibility certificate tests off")
    ap.add_argument("--polish", action="store_true",
                    help="sparse workloads: feasibility polishing after the optimal solve")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy three times (counter calibration)")
    ap.add_argument("--workload", default="sparse",
                    choices=["sparse", "sparse-infeasible", "dense", "dense-knapsack", "batch-grid",
                             "batch-ragged",
                             "learn-grid", "spo-grid", "qp-portfolio"],
                    help="sparse (default, the headline line); sparse-infeasible: the same LP "
                         "with one equality row duplicated at a moved right-hand side, solved "
                         "until its infeasibility certificate; dense 20k x 40k, "
                         "batched grid min-cost flows (2,048 x 32x32 grid) or the ragged batch "
                         "(1,024 planted LPs); the batched modes also time the plain solver "
                         "looped one instance at a time on a subset; learn-grid: training steps "
                         "of the shortest-path cost model through 1,000 unrolled iterations "
                         "(256 grids); spo-grid: SPO+ training steps on the same grids (batched "
                         "solves to 1e-4, warm-started); qp-portfolio: 512 portfolio QPs, solve "
                         "and unrolled gradient")
    ap.add_argument("--batch", type=int, default=0, help="batch size override (batched modes)")
    ap.add_argument("--threads", type=int, default=0,
                    help="threads per instance of the batch solves (default: the library's choice)")
    ap.add_argument("--layout", default="",
                    help="sparse workloads: product-layout options of the solver as "
                         "key=value,... (panel_rows, panel_min_len, panel_wgs, hot_cols)")
    ap.add_argument("--loop-sample", type=int, default=16,
                    help="instances solved one at a time for the looped comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(every workload here, batched ones included, runs on a single MI355X)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copied 3 x 1 GiB")
        return

    import gen
    from paper_2412_09734_amd import Solver

    if args.workload in ("batch-grid", "batch-ragged"):
        return bench_batch(args)
    if args.workload == "dense":
        return bench_dense(args)
    if args.workload == "dense-knapsack":
        return bench_knapsack(args)
    if args.workload == "learn-grid":
        return bench_learn(args)
    if args.workload == "spo-grid":
        return bench_spo(args)
    if args.workload == "qp-portfolio":
        return bench_qp(args)

    log(f"bench: generating sparse LP m={args.m} n={args.n}")
    t = time.perf_counter()
    lp = gen.large_zipf_lp(m=args.m, n=args.n, seed=gen.seed_for(1, 0))
    log(f"bench: nnz={lp.nnz} generated in {time.perf_counter() - t:.1f} s")
    infeasible = args.workload == "sparse-infeasible"
    if infeasible:
        lp = gen.contradict_row(lp, seed=1)
        log(f"bench: duplicated equality row {lp.meta['row']} with its right-hand side moved by 1")
    dev = torch.device("cuda:0")
    data = dict(rowptr=torch.from_numpy(lp.rowptr).to(dev), colidx=torch.from_numpy(lp.colidx).to(dev),
                val=torch.from_numpy(lp.val).to(dev), c=torch.from_numpy(lp.c).to(dev),
                lc=torch.from_numpy(lp.lc).to(dev), uc=torch.from_numpy(lp.uc).to(dev),
                lv=torch.from_numpy(lp.lv).to(dev), uv=torch.from_numpy(lp.uv).to(dev))
    torch.cuda.synchronize()

    extra = {"iteration_limit": args.iteration_limit} if args.iteration_limit > 0 else {}
    if args.polish:
        extra["feasibility_polishing"] = 1
    if args.eps != 1e-4:
        extra["eps"] = args.eps
    for kv in filter(None, args.layout.split(",")):
        k, v = kv.split("=")
        if k not in ("panel_rows", "panel_min_len", "panel_wgs", "hot_cols"):
            raise SystemExit(f"unknown layout option {k}")
        extra[k] = int(v)

    def step(timing_chunk=-1):
        with Solver(lp.m, lp.n, device=dev, timing_chunk=timing_chunk, **extra, **data) as s:
            x, y, info = s.solve()
        return info

    for w in range(args.warmup):
        info = step()
        log(f"bench: warmup {w}: {info['status_name']} iters={info['iterations']} "
            f"setup={info['setup_seconds']:.3f}s solve={info['solve_seconds']:.3f}s kkt={info['kkt_rel']:.2e}")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        infos.append(step(timing_chunk=2))
        log(f"bench: step {k}: {infos[-1]['status_name']} iters={infos[-1]['iterations']} "
            f"solve={infos[-1]['solve_seconds']:.3f}s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    last = infos[-1]
    iters = int(last["iterations"])
    kb = kernel_bytes(lp.m, lp.n, lp.nnz)
    samples = [i for i in infos if i["kernel_samples"] > 0]
    prim_ms = float(np.mean([i["kernel_primal_ms"] for i in samples])) if samples else float("nan")
    dual_ms = float(np.mean([i["kernel_dual_ms"] for i in samples])) if samples else float("nan")
    dom = "primal" if prim_ms >= dual_ms else "dual"
    other = "dual" if dom == "primal" else "primal"
    ms = {"primal": prim_ms, "dual": dual_ms}
    achieved = kb[dom] / (ms[dom] * 1e-3) / 1e9
    iter_bytes = kb["primal"] + kb["dual"]
    iter_ms = prim_ms + dual_ms
    solve_s = float(np.mean([i["solve_seconds"] for i in infos]))
    setup_s = float(np.mean([i["setup_seconds"] for i in infos]))
    # the library's automatic layouts for a large sparse A (options panel_rows / hot_cols)
    layout = dict(kv.split("=") for kv in filter(None, args.layout.split(",")))
    panels = layout.get("panel_rows", "-1") != "0" and (lp.m > 262144 or int(layout.get("panel_rows", "-1")) > 0)
    hot = layout.get("hot_cols", "-1") != "0" and (lp.n > 262144 or int(layout.get("hot_cols", "-1")) > 0)
    names = {"primal": ("primal step: k_panel_dot (long rows of A~', LDS panels of y) beside k_primal_sell "
                        "(SELL-64 rows) on a second stream, then k_primal_panels (panel sums + primal update)"
                        if panels else "k_primal"),
             "dual": "k_dual_hot (x_ext[0, 20480) in LDS)" if hot else "k_dual"}
    full_size = (lp.m, lp.n) == (1_000_000, 2_000_000) and not args.layout
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom) if full_size else None,
            "kernel": names[dom],
            "algorithmic_bytes_per_launch": kb[dom], "avg_launch_ms": round(ms[dom], 5),
            "other_step": {"kernel": names[other], "algorithmic_bytes": kb[other],
                           "avg_ms": round(ms[other], 5),
                           "achieved": round(kb[other] / (ms[other] * 1e-3) / 1e9, 1),
                           "traffic": measured_traffic(other) if full_size else None},
            "iteration_gbps": round(iter_bytes / (iter_ms * 1e-3) / 1e9, 1)}
    out = {
        "metric": METRIC, "value": round(args.steps / elapsed, 5), "unit": "LPs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"plain r2HPDHG to an infeasibility certificate, sparse LP m={lp.m} "
                                f"n={lp.n} Zipf columns with one contradicting row" if infeasible else
                                f"plain r2HPDHG, sparse planted LP m={lp.m} n={lp.n} Zipf columns"),
                   "status": last["status_name"],
                   "feasibility_polishing": bool(args.polish),
                   "polish_iterations": int(last["polish_iterations"]),
                   "rel_primal": last["rel_primal_res"], "rel_dual": last["rel_dual_res"],
                   "rel_gap": last["rel_gap"],
                   "m": lp.m, "n": lp.n, "nnz": int(lp.nnz), "eps": args.eps,
                   "iterations": iters, "restarts": int(last["restarts"]),
                   "power_iters": int(last["power_iters"]), "kkt_rel": last["kkt_rel"],
                   "primal_obj": last["primal_obj"], "planted_obj": lp.v_star,
                   "setup_s": round(setup_s, 4), "solve_s": round(solve_s, 4),
                   "iter_us_kernels": round(iter_ms * 1e3, 2),
                   "iter_us_wall": round(solve_s / iters * 1e6, 2),
                   "primal_kernel_ms": round(prim_ms, 5), "dual_kernel_ms": round(dual_ms, 5),
                   "bytes_per_iteration": iter_bytes},
        "roofline": roof,
    }
    sp = stream_peak()
    roof["stream_gbs"] = sp
    roof["frac_of_stream"] = round(achieved / max(sp.values()), 4)
    if not args.no_batched and not infeasible:
        log("bench: batched grid LPs vs the plain solver looped")
        out["config"]["batched"] = batched_vs_plain()
    if not args.no_other and not infeasible and not args.layout and not args.iteration_limit:
        log("bench: 512 portfolio QPs (batched solve and unrolled gradient)")
        out["config"]["qp_portfolio"] = qp_portfolio_run(512, steps=3, warmup=1, envelope=False)
        log("bench: dense knapsack shape, first 10,000 iterations")
        out["config"]["dense_knapsack"] = knapsack_run(steps=1, warmup=1)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(lp, iters, int(last["power_iters"]))
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Batched LPs in one persistent launch vs the plain solver looped one
    instance at a time (same MI355X). value = LPs solved per second."""
    import numpy as np
    import torch

    import gen
    from paper_2412_09734_amd.solver import BatchSolver, Solver

    dev = torch.device("cuda:0")

    def resident(kw):
        # problem arrays copied to the device once; every step creates the batch
        # (layout, scaling, power iteration) from device memory and solves it
        out = {}
        for k, v in kw.items():
            if isinstance(v, np.ndarray) and k not in ("row_off", "col_off"):
                dt = torch.int32 if v.dtype.kind in "iu" else torch.float64
                out[k] = torch.from_numpy(np.ascontiguousarray(v)).to(dev, dt)
            else:
                out[k] = v
        return out

    if args.workload == "batch-grid":
        B = args.batch or 2048
        sb = gen.grid_mincost_batch(batch=B, seed=gen.seed_for(3, 0))
        kw = resident(dict(shared_a=True, batch=B, m=sb.m, n=sb.n, rowptr=sb.rowptr, colidx=sb.colidx,
                           val=sb.val, c=sb.c, lc=sb.lc, uc=sb.uc, lv=sb.lv, uv=sb.uv))
        inst = [sb.instance(b) for b in range(min(args.loop_sample, B))]
        name = f"batched r2HPDHG, {B} min-cost-flow LPs sharing a 32x32 grid incidence (1024 x 3968)"
    else:
        B = args.batch or 1024
        lps = gen.ragged_planted_batch(batch=B, seed=gen.seed_for(3, 500))
        kw = resident(BatchSolver.ragged_arrays(lps))
        inst = lps[: min(args.loop_sample, B)]
        name = f"batched r2HPDHG, {B} planted LPs m~U{{50..500}}, n=2m, 5% density"
    torch.cuda.synchronize()
    if args.no_infeasibility_tests:
        kw = dict(kw, eps_primal_infeasible=0.0, eps_dual_infeasible=0.0)
    make = lambda: BatchSolver(**kw)  # noqa: E731
    with make() as bs:
        best = bs.autotune(128)
        log(f"bench: autotuned threads per instance = {best}")
    torch.cuda.synchronize()
    for w in range(args.warmup):
        with make() as bs:
            bs.set_launch(best)
            bs.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_create = t_solve = 0.0
    for _ in range(args.steps):
        ta = time.perf_counter()
        with make() as bs:
            torch.cuda.synchronize()
            tb = time.perf_counter()
            bs.set_launch(best)
            x, y, res = bs.solve()
            torch.cuda.synchronize()
            t_solve += time.perf_counter() - tb
        t_create += tb - ta
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    solved = sum(r["status"] == 1 for r in res)
    iters = [r["iterations"] for r in res]
    # plain solver, one instance at a time (create + solve each)
    t1 = time.perf_counter()
    loop_ok = 0
    for lp in inst:
        with Solver.from_lp(lp) as s:
            _, _, r = s.solve()
        loop_ok += r["status"] == 1
    torch.cuda.synchronize()
    loop_rate = len(inst) / (time.perf_counter() - t1)
    out = {"metric": METRIC, "value": round(args.steps * solved / el, 2), "unit": "LPs/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(el / args.steps * 1e3, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": name, "batch": B, "threads_per_instance": best,
                      "solved": int(solved), "iterations_mean": float(np.mean(iters)),
                      "iterations_max": int(np.max(iters)),
                      "create_ms": round(t_create / args.steps * 1e3, 2),
                      "solve_ms": round(t_solve / args.steps * 1e3, 2),
                      "plain_looped_lps_per_s": round(loop_rate, 3),
                      "plain_looped_sample": len(inst), "plain_looped_solved": int(loop_ok),
                      "speedup_vs_plain_looped": round(args.steps * solved / el / loop_rate, 1)}}
    print(json.dumps(out), flush=True)


def bench_dense(args):
    """Plain r2HPDHG on the dense 20,000 x 40,000 LP (6.4 GB row-major)."""
    import numpy as np
    import torch

    import gen
    from paper_2412_09734_amd import Solver

    lp = gen.dense_planted_lp(seed=gen.seed_for(2, 0))
    dev = torch.device("cuda:0")
    a = torch.from_numpy(lp.dense).to(dev)
    vec = {k: torch.from_numpy(getattr(lp, k)).to(dev) for k in ("c", "lc", "uc", "lv", "uv")}
    torch.cuda.synchronize()
    extra = {"iteration_limit": args.iteration_limit} if args.iteration_limit > 0 else {}

    def step(timing_chunk=-1):
        with Solver(lp.m, lp.n, None, None, None, a_dense=a, device=dev, timing_chunk=timing_chunk,
                    **extra, **vec) as s:
            return s.solve()[2]

    for w in range(args.warmup):
        info = step()
        log(f"bench: warmup {w}: {info['status_name']} iters={info['iterations']} solve={info['solve_seconds']:.2f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step(timing_chunk=2) for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    last = infos[-1]
    total = lp.m * lp.n
    kb_rows = 8 * total + 8 * (lp.n + 5 * lp.m)
    kb_cols = 8 * total + 8 * (lp.m + 7 * lp.n)
    prim = float(np.mean([i["kernel_primal_ms"] for i in infos if i["kernel_samples"]] or [np.nan]))
    dual = float(np.mean([i["kernel_dual_ms"] for i in infos if i["kernel_samples"]] or [np.nan]))
    roof = {"bound": "hbm", "achieved": round(kb_rows / (dual * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(kb_rows / (dual * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": None, "kernel": "k_dense_rows<ROW_DUAL>", "algorithmic_bytes_per_launch": kb_rows,
            "avg_launch_ms": round(dual, 4),
            "column_pass_gbps": round(kb_cols / (prim * 1e-3) / 1e9, 1)}
    sp = stream_peak()
    roof["stream_gbs"] = sp
    roof["frac_of_stream"] = round(kb_rows / (dual * 1e-3) / 1e9 / max(sp.values()), 4)
    out = {"metric": METRIC, "value": round(args.steps / el, 5), "unit": "LPs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "plain r2HPDHG, dense planted LP 20000 x 40000", "iterations": last["iterations"],
                      "status": last["status_name"], "kkt_rel": last["kkt_rel"],
                      "primal_obj": last["primal_obj"], "planted_obj": lp.v_star,
                      "iter_ms_kernels": round(prim + dual, 4)},
           "roofline": roof}
    print(json.dumps(out), flush=True)


def knapsack_run(steps: int, warmup: int, limit: int = 10_000) -> dict:
    """The paper's hardware-comparison protocol on the dense knapsack shape
    (1,000 x 100,000, FP64): the time of the first `limit` iterations (the
    tolerance is set unreachably small so every run hits the limit)."""
    import numpy as np
    import torch

    import gen
    from paper_2412_09734_amd import Solver

    lp = gen.dense_knapsack_lp(seed=gen.seed_for(2, 500))
    dev = torch.device("cuda:0")
    a = torch.from_numpy(lp.dense).to(dev)
    vec = {k: torch.from_numpy(getattr(lp, k)).to(dev) for k in ("c", "lc", "uc", "lv", "uv")}
    torch.cuda.synchronize()

    def step(timing_chunk=-1):
        with Solver(lp.m, lp.n, None, None, None, a_dense=a, device=dev, timing_chunk=timing_chunk,
                    iteration_limit=limit, eps=1e-14, **vec) as s:
            return s.solve()[2]

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    infos = [step(timing_chunk=2) for _ in range(steps)]
    del a
    solve = float(np.mean([i["solve_seconds"] for i in infos]))
    setup = float(np.mean([i["setup_seconds"] for i in infos]))
    last = infos[-1]
    prim = float(np.mean([i["kernel_primal_ms"] for i in infos if i["kernel_samples"]] or [np.nan]))
    dual = float(np.mean([i["kernel_dual_ms"] for i in infos if i["kernel_samples"]] or [np.nan]))
    pass_bytes = 8 * lp.m * lp.n
    return {"workload": f"plain r2HPDHG, dense knapsack LP {lp.m} x {lp.n}, {last['iterations']} iterations",
            "solve_s": round(solve, 4), "setup_s": round(setup, 4),
            "iter_us": round(solve / max(1, last["iterations"]) * 1e6, 2),
            "row_pass_gbps": round(pass_bytes / (dual * 1e-3) / 1e9, 1),
            "column_pass_gbps": round(pass_bytes / (prim * 1e-3) / 1e9, 1),
            "paper_context_h200_fp64_s": 4.15}


def bench_knapsack(args):
    r = knapsack_run(args.steps, args.warmup, args.iteration_limit or 10_000)
    solve = r.pop("solve_s")
    out = {"metric": "seconds for the first 10,000 iterations (dense knapsack shape)",
           "value": solve, "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(solve * 1e3, 2), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": r}
    print(json.dumps(out), flush=True)


def bench_learn(args):
    """One training step of the shortest-path cost model: c_hat = f W on the
    device, 1,000 unrolled iterations of the batch, regret under the true
    costs, reverse pass, weight gradient (all in libpdhg kernels), then a
    host-side gradient step on the 5 weights. value = LPs differentiated per
    second (batch / step time)."""
    import numpy as np
    import torch

    import gen
    from paper_2412_09734_amd import heads
    from paper_2412_09734_amd.solver import BatchSolver

    B = args.batch or 256
    T = 1000
    sb, f, w_star, W = gen.shortest_path_learning(batch=B, seed=gen.seed_for(4, 0))
    dev = torch.device("cuda:0")
    fd = torch.from_numpy(f).to(dev)
    ct = torch.from_numpy(sb.c).to(dev)
    with BatchSolver.from_shared(sb, eps=1e-8) as bs:
        _, _, res = bs.solve()                       # optimal values under the true costs
    vstar = torch.tensor([r["primal_obj"] for r in res], dtype=torch.float64, device=dev)
    lr = 0.05
    with BatchSolver.from_shared(sb, threads=args.threads or None) as bs:
        def step(Wv):
            chat = heads.linear_costs(fd, Wv)
            bs.update_data(c=chat)
            x, _ = bs.unrolled(T)
            loss = heads.regret(ct, x, vstar)
            gc = bs.backward(ct)[0]
            gW = heads.linear_costs_backward(fd, gc)
            return float(loss.mean()), gW.cpu().numpy() / B
        for _ in range(args.warmup):
            step(W)
        torch.cuda.synchronize()
        losses = []
        t0 = time.perf_counter()
        for k in range(args.steps):
            l, g = step(W)
            W = W - lr * g
            losses.append(l)
            log(f"bench: learn step {k}: mean regret {l:.4f}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    out = {"metric": METRIC, "value": round(args.steps * B / el, 2), "unit": "LPs/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(el / args.steps * 1e3, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"learning step: {B} grid shortest-path LPs (32x32), linear cost "
                                  f"model on 5 features, {T} unrolled r2HPDHG iterations + reverse pass",
                      "batch": B, "unrolled_iterations": T, "mean_regret_first": losses[0],
                      "mean_regret_last": losses[-1]}}
    print(json.dumps(out), flush=True)


def bench_spo(args):
    """One SPO+ training step of the shortest-path cost model: c_hat = f W,
    inner costs 2 c_hat - c, one batched solve to 1e-4 warm-started from the
    previous step's primal and dual solutions, SPO+ loss and subgradient, weight gradient (all
    in libpdhg kernels), then a host-side gradient step (rate 1e-4) on the 5
    weights.
    value = LPs solved and differentiated per second (batch / step time)."""
    import numpy as np
    import torch

    import gen
    from paper_2412_09734_amd import heads
    from paper_2412_09734_amd.solver import BatchSolver

    B = args.batch or 256
    sb, f, _, W = gen.shortest_path_learning(batch=B, seed=gen.seed_for(4, 0))
    dev = torch.device("cuda:0")
    fd = torch.from_numpy(f).to(dev)
    ct = torch.from_numpy(sb.c).to(dev)
    with BatchSolver.from_shared(sb, eps=1e-8) as bs:
        w_star, _, res = bs.solve()                  # optimal decisions under the true costs
    z_star = torch.tensor([r["primal_obj"] for r in res], dtype=torch.float64, device=dev)
    lr = 1e-4   # larger plain-gradient steps diverge: the subgradient sums over ~4,000 arcs
    off = dict(eps_primal_infeasible=0.0, eps_dual_infeasible=0.0) if args.no_infeasibility_tests else {}
    with BatchSolver.from_shared(sb, threads=args.threads or None, **off) as bs:
        if not args.threads:
            bs.update_data(c=heads.spo_plus_costs(heads.linear_costs(fd, W), ct))
            log(f"bench: autotuned threads per instance = {bs.autotune(128)}")
        prev = [None, None]

        def step(Wv):
            chat = heads.linear_costs(fd, Wv)
            bs.update_data(c=heads.spo_plus_costs(chat, ct))
            wt, yt, r = bs.solve(x_init=prev[0], y_init=prev[1])
            prev[0], prev[1] = wt, yt
            loss, g = heads.spo_plus(chat, ct, w_star, z_star, wt)
            gW = heads.linear_costs_backward(fd, g)
            return float(loss.mean()), gW.cpu().numpy() / B, r
        # warm-up steps are training steps too: the timed steps never re-solve
        # the costs their warm start came from
        for _ in range(args.warmup):
            _, g, _ = step(W)
            W = W - lr * g
        torch.cuda.synchronize()
        losses, iters = [], []
        t0 = time.perf_counter()
        for k in range(args.steps):
            l, g, r = step(W)
            W = W - lr * g
            losses.append(l)
            iters.append(float(np.mean([q["iterations"] for q in r])))
            log(f"bench: SPO+ step {k}: mean loss {l:.4f}, mean iterations {iters[-1]:.0f}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    out = {"metric": METRIC, "value": round(args.steps * B / el, 2), "unit": "LPs/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(el / args.steps * 1e3, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"SPO+ learning step: {B} grid shortest-path LPs (32x32), linear cost "
                                  "model on 5 features, batched solves to 1e-4 warm-started",
                      "batch": B, "mean_iterations": iters, "mean_spo_loss_first": losses[0],
                      "mean_spo_loss_last": losses[-1]}}
    print(json.dumps(out), flush=True)


def qp_portfolio_run(B: int, steps: int, warmup: int, envelope: bool = True) -> dict:
    """B portfolio QPs (n=500, Q = F F' + diag d, F shared, rank 20):
    batched rAPDHG solve to 1e-4 (QPs/s), then 1,000 unrolled iterations with
    the reverse pass for the gradient of the value in (c, d)."""
    import numpy as np
    import torch

    import gen
    from paper_2412_09734_amd import heads
    from paper_2412_09734_amd.solver import BatchSolver
    from types import SimpleNamespace

    T = 1000
    p = gen.portfolio_qp_batch(batch=B, seed=gen.seed_for(4, 500))
    sb = SimpleNamespace(m=p["m"], n=p["n"], rowptr=p["rowptr"], colidx=p["colidx"], val=p["val"],
                         c=p["c"], lc=np.tile(p["lc"], (B, 1)), uc=np.tile(p["uc"], (B, 1)),
                         lv=np.tile(p["lv"], (B, 1)), uv=np.tile(p["uv"], (B, 1)),
                         q_factor=p["F"], q_diag=p["d"])
    dev = torch.device("cuda:0")
    out = {"workload": f"batched rAPDHG, {B} portfolio QPs n=500, Q = F F' + diag(d), F rank 20 shared",
           "batch": B}
    with BatchSolver.from_shared(sb) as bs:
        for _ in range(warmup):
            bs.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x, y, res = bs.solve()
        torch.cuda.synchronize()
        t_solve = (time.perf_counter() - t0) / steps
        solved = sum(r["status"] == 1 for r in res)
        iters = [r["iterations"] for r in res]
        Fd = torch.from_numpy(p["F"]).to(dev)
        dd = torch.from_numpy(p["d"]).to(dev)
        cd = torch.from_numpy(p["c"]).to(dev)
        for _ in range(warmup):
            xT, _ = bs.unrolled(T)
            val, gx = heads.qp_value(Fd, dd, cd, xT)
            bs.backward(gx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            xT, _ = bs.unrolled(T)
            val, gx = heads.qp_value(Fd, dd, cd, xT)
            gc, _, _, gd = bs.backward(gx)
        torch.cuda.synchronize()
        t_grad = (time.perf_counter() - t1) / steps
        out.update({"solve_ms": round(t_solve * 1e3, 3), "qps_per_s": round(solved / t_solve, 2),
                    "solved": int(solved), "iterations_mean": float(np.mean(iters)),
                    "iterations_max": int(np.max(iters)), "unrolled_iterations": T,
                    "grad_ms": round(t_grad * 1e3, 2), "qps_per_s_with_gradient": round(B / t_grad, 2)})
        if envelope:
            # envelope check (untimed): dV/dc = x* with x* from a batched solve
            # to relative KKT 1e-10, over the instances that solve converges
            # within T iterations (the unrolled point has converged there too)
            with BatchSolver.from_shared(sb, eps=1e-10, iteration_limit=100000) as tight:
                xs_t, _, res_t = tight.solve()
            conv = np.array([r["status"] == 1 and r["iterations"] < T for r in res_t])
            gc_tot = (gc + xT).cpu().numpy()
            err = np.abs(gc_tot - xs_t.cpu().numpy()).max(axis=1)
            out.update({"envelope_c_max_abs_err": float(err[conv].max()) if conv.any() else None,
                        "envelope_instances": int(conv.sum()),
                        "envelope_reference": "batched solve to relative KKT 1e-10"})
    return out


def bench_qp(args):
    r = qp_portfolio_run(args.batch or 512, args.steps, args.warmup)
    t_solve = r["solve_ms"] * 1e-3
    out = {"metric": METRIC, "value": r.pop("qps_per_s"), "unit": "QPs/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(t_solve * 1e3, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": r}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
