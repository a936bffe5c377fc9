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


def cpu_baseline(lp, gpu_iters: int, gpu_power_iters: int) -> dict:
    """The oracle on a bounded sample of the same LP: its scaling, then 65
    iterations (checks at the first and last), timed on one host core; the
    per-LP time is extrapolated to the GPU's power-iteration and iteration
    counts (each power step costs about one iteration's two products)."""
    import oracle
    oracle.build(force=False)
    sample_iters = 65
    t0 = time.perf_counter()
    orc = oracle.Oracle(lp, power_max_iters=1, iteration_limit=sample_iters)
    t_setup = time.perf_counter() - t0
    t1 = time.perf_counter()
    orc.solve()
    t_iter = (time.perf_counter() - t1) / sample_iters
    orc.close()
    per_lp = t_setup + (gpu_power_iters + gpu_iters) * t_iter
    return {"value": 1.0 / per_lp, "unit": "LPs/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle scaling ({t_setup:.2f} s) + {sample_iters} iterations "
                       f"({t_iter * 1e3:.1f} ms each) on the full LP, extrapolated to "
                       f"{gpu_power_iters} power steps + {gpu_iters} iterations per LP")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=1_000_000)
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iteration-limit", type=int, default=0,
                    help="stop every solve after this many iterations (profiling runs only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the batched and sharded paths run on a single MI355X in this build)",
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

    log(f"bench: generating sparse LP m={args.m} n={args.n}")
    t = time.perf_counter()
    lp = gen.large_zipf_lp(m=args.m, n=args.n, seed=gen.seed_for(1, 0))
    log(f"bench: nnz={lp.nnz} generated in {time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    data = dict(rowptr=torch.from_numpy(lp.rowptr).to(dev), colidx=torch.from_numpy(lp.colidx).to(dev),
                val=torch.from_numpy(lp.val).to(dev), c=torch.from_numpy(lp.c).to(dev),
                lc=torch.from_numpy(lp.lc).to(dev), uc=torch.from_numpy(lp.uc).to(dev),
                lv=torch.from_numpy(lp.lv).to(dev), uv=torch.from_numpy(lp.uv).to(dev))
    torch.cuda.synchronize()

    extra = {"iteration_limit": args.iteration_limit} if args.iteration_limit > 0 else {}

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
    dom_ms = max(prim_ms, dual_ms)
    achieved = kb[dom] / (dom_ms * 1e-3) / 1e9
    iter_bytes = kb["primal"] + kb["dual"]
    iter_ms = prim_ms + dual_ms
    solve_s = float(np.mean([i["solve_seconds"] for i in infos]))
    setup_s = float(np.mean([i["setup_seconds"] for i in infos]))
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_primal" if dom == "primal" else "k_dual",
            "algorithmic_bytes_per_launch": kb[dom], "avg_launch_ms": round(dom_ms, 5),
            "iteration_gbps": round(iter_bytes / (iter_ms * 1e-3) / 1e9, 1)}
    out = {
        "metric": METRIC, "value": round(args.steps / elapsed, 5), "unit": "LPs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"plain r2HPDHG, sparse planted LP m={lp.m} n={lp.n} Zipf columns",
                   "m": lp.m, "n": lp.n, "nnz": int(lp.nnz), "eps": 1e-4,
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
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(lp, iters, int(last["power_iters"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
