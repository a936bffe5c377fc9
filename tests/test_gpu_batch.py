"""GPU parity of the batched solver (one persistent launch): every instance
against the CPU oracle and against the plain GPU solver on that instance."""

import sys

import numpy as np
import pytest

import gen
from gpu_util import rel_inf, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pdhg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_09734_amd.solver as s
    return s


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _close(a, b, tol=1e-6):
    return abs(a - b) <= tol * (1 + abs(b))


def test_shared_grid_batch_matches_oracle_and_plain(pdhg, oracle_lib):
    """n = 528 columns: the default launch (1024 threads, one column per
    thread), 256 and 128 threads (4 and 8 columns per thread on chip) and 64
    threads (memory-resident kernel) all reach the oracle's optimum."""
    _say("case: shared-A batch, 12x12 grid min-cost flow, B=24")
    sb = gen.grid_mincost_batch(batch=24, rows=12, cols=12, seed=3100)
    ref = []
    for b in range(sb.batch):
        lp = sb.instance(b)
        _, _, ro = oracle_lib.Oracle(lp).solve()
        with pdhg.Solver.from_lp(lp) as s:
            _, _, rp = s.solve()
        ref.append((lp, ro, rp))
    sc = oracle_lib.Oracle(ref[0][0]).scaling()   # the instances share A
    for threads in (None, 256, 128, 64):
        _say(f"  threads per instance: {threads or 'default'}")
        with pdhg.BatchSolver.from_shared(sb, threads=threads) as bs:
            x, y, res = bs.solve()
        for b, (lp, ro, rp) in enumerate(ref):
            rb = res[b]
            assert rb["status_name"] == "optimal" and rb["kkt_rel"] <= 1e-4, (threads, b, rb)
            assert rb["power_iters"] == sc["power_iters"], (rb["power_iters"], sc["power_iters"])
            assert abs(rb["eta"] - sc["eta"]) <= 1e-10 * sc["eta"], (rb["eta"], sc["eta"])
            assert _close(rb["primal_obj"], ro["primal_obj"]), (threads, b, rb["primal_obj"], ro["primal_obj"])
            assert _close(rb["primal_obj"], rp["primal_obj"]), (threads, b, rb["primal_obj"], rp["primal_obj"])
            kb = oracle_lib.kkt(lp, to_np(x[b]), to_np(y[b]))
            assert kb["kkt"] <= 1e-4 * (1 + 1e-6)
        _say(f"  iterations: {[r['iterations'] for r in res[:8]]}")


@pytest.mark.parametrize("threads", [None, 256])
def test_ragged_batch_matches_oracle(pdhg, oracle_lib, threads):
    """n <= 294 columns per instance: one column per thread at the default
    launch, two at 256 threads."""
    _say(f"case: ragged batch of planted LPs, B=12, m in 50..150, threads {threads or 'default'}")
    lps = gen.ragged_planted_batch(batch=12, m_lo=50, m_hi=150, seed=3600)
    with pdhg.BatchSolver.from_lps(lps, threads=threads) as bs:
        x, y, res = bs.solve()
        for b, lp in enumerate(lps):
            orc = oracle_lib.Oracle(lp)
            sc = orc.scaling()
            _, _, ro = orc.solve()
            cs, rs = bs.instance_slices(b)
            rb = res[b]
            assert rb["status_name"] == "optimal", (b, rb)
            assert rb["power_iters"] == sc["power_iters"], (b, rb["power_iters"], sc["power_iters"])
            assert abs(rb["eta"] - sc["eta"]) <= 1e-10 * sc["eta"], (b, rb["eta"], sc["eta"])
            assert _close(rb["primal_obj"], ro["primal_obj"]), (b, rb["primal_obj"], ro["primal_obj"])
            assert rb["iterations"] == ro["iterations"], (b, rb["iterations"], ro["iterations"])
            kb = oracle_lib.kkt(lp, to_np(x[cs]), to_np(y[rs]))
            assert abs(kb["kkt"] - rb["kkt_rel"]) <= 1e-9 + 1e-6 * kb["kkt"]


def test_ragged_batch_beyond_lds_matches_oracle(pdhg, oracle_lib):
    """Instances whose gathered vectors exceed the on-chip budget (n + m >
    8192) run the memory-resident kernel; a small instance in the same batch
    does not change that choice."""
    _say("case: ragged batch with m ~ 3000, n ~ 6000 instances (memory-resident kernel)")
    lps = gen.ragged_planted_batch(batch=2, m_lo=2900, m_hi=3000, density=0.003, seed=3950)
    lps.append(gen.ragged_planted_batch(batch=1, m_lo=60, m_hi=60, seed=3951)[0])
    assert max(lp.m + lp.n for lp in lps) > 8192
    with pdhg.BatchSolver.from_lps(lps) as bs:
        x, y, res = bs.solve()
        for b, lp in enumerate(lps):
            orc = oracle_lib.Oracle(lp)
            sc = orc.scaling()
            _, _, ro = orc.solve()
            cs, rs = bs.instance_slices(b)
            rb = res[b]
            assert rb["status_name"] == "optimal", (b, rb)
            assert rb["power_iters"] == sc["power_iters"], (b, rb["power_iters"], sc["power_iters"])
            assert abs(rb["eta"] - sc["eta"]) <= 1e-10 * sc["eta"], (b, rb["eta"], sc["eta"])
            assert _close(rb["primal_obj"], ro["primal_obj"]), (b, rb["primal_obj"], ro["primal_obj"])
            assert rb["iterations"] == ro["iterations"], (b, rb["iterations"], ro["iterations"])
            kb = oracle_lib.kkt(lp, to_np(x[cs]), to_np(y[rs]))
            assert abs(kb["kkt"] - rb["kkt_rel"]) <= 1e-9 + 1e-6 * kb["kkt"]


def test_batch_determinism_and_launch_shapes(pdhg):
    _say("case: batch determinism across launches and thread counts")
    sb = gen.grid_mincost_batch(batch=40, rows=8, cols=8, seed=3200)
    with pdhg.BatchSolver.from_shared(sb) as bs:
        x1, y1, r1 = bs.solve()
        x1 = to_np(x1)
        x2, y2, r2 = bs.solve()
        np.testing.assert_array_equal(x1, to_np(x2))
        objs = {}
        for t in (64, 128, 256, 512):
            bs.set_launch(t, workgroups=7)
            _, _, r = bs.solve()
            objs[t] = [q["primal_obj"] for q in r]
        best = bs.autotune(64)
        assert best in (64, 128, 256, 512, 1024)
    for t, o in objs.items():
        for a, b in zip(o, [q["primal_obj"] for q in r1]):
            assert _close(a, b), (t, a, b)


def test_batch_iteration_limit(pdhg, oracle_lib):
    _say("case: batch iteration limit")
    lps = gen.ragged_planted_batch(batch=4, m_lo=40, m_hi=60, seed=3700)
    with pdhg.BatchSolver.from_lps(lps, iteration_limit=70) as bs:
        x, y, res = bs.solve()
        for b, lp in enumerate(lps):
            xo, yo, ro = oracle_lib.Oracle(lp, iteration_limit=70).solve()
            cs, rs = bs.instance_slices(b)
            assert res[b]["iterations"] == 70 and res[b]["status"] == 4
            assert np.abs(to_np(x[cs]) - xo).max() <= 1e-10 * max(1.0, np.abs(xo).max())


def _mixed_batch():
    """Planted feasible LPs with infeasible and unbounded ones among them."""
    lps = gen.ragged_planted_batch(batch=6, m_lo=40, m_hi=90, seed=3990)
    lps.insert(1, gen.infeasible_lp("duplicate_row", 60, 120, seed=0))
    lps.insert(3, gen.infeasible_lp("unbounded", 60, 120, seed=2))
    lps.insert(5, gen.infeasible_lp("boxed_sum", 30, 50, seed=3))
    lps.append(gen.infeasible_lp("unbounded", 300, 600, seed=1))   # n > 8 x 64: memory-resident at 64 threads
    return lps


@pytest.mark.parametrize("threads", [None, 64])
def test_batch_infeasibility_matches_oracle(pdhg, oracle_lib, threads):
    """Each instance of a mixed batch ends as the oracle ends it (status and
    iteration count), and a certifying ray comes back in its output slice;
    64 threads per instance run the memory-resident kernel for the largest."""
    _say(f"case: mixed ragged batch with infeasible / unbounded instances, threads {threads or 'default'}")
    lps = _mixed_batch()
    with pdhg.BatchSolver.from_lps(lps, threads=threads, iteration_limit=100000) as bs:
        x, y, res = bs.solve()
        for b, lp in enumerate(lps):
            xo, yo, ro = oracle_lib.Oracle(lp, iteration_limit=100000).solve()
            cs, rs = bs.instance_slices(b)
            rb = res[b]
            assert rb["status_name"] == ro["status_name"], (b, rb["status_name"], ro["status_name"])
            assert rb["iterations"] == ro["iterations"], (b, rb["iterations"], ro["iterations"])
            if ro["status_name"] == "primal_infeasible":
                assert rel_inf(to_np(y[rs]), yo) <= 1e-8
            elif ro["status_name"] == "dual_infeasible":
                assert rel_inf(to_np(x[cs]), xo) <= 1e-8
            else:
                assert ro["status_name"] == "optimal"
                assert _close(rb["primal_obj"], ro["primal_obj"])


def test_batch_infeasibility_switched_off(pdhg):
    _say("case: mixed batch with the infeasibility tests off (lean kernels)")
    lps = _mixed_batch()
    with pdhg.BatchSolver.from_lps(lps, iteration_limit=3000, eps_primal_infeasible=0.0,
                                   eps_dual_infeasible=0.0) as bs:
        _, _, res = bs.solve()
    names = [r["status_name"] for r in res]
    assert names[1] == names[3] == names[5] == names[-1] == "iteration_limit", names
    assert names[0] == names[2] == names[4] == "optimal", names


def _grid_with_certificates(rows, cols, seed):
    """Six grid min-cost flows sharing A: instance 1 is primal infeasible
    (supply 200 at its source, more than the <= 4 x 20 capacity leaving any
    node) and instance 3 unbounded (both arcs between two nodes cost -1 and
    have no capacity, so flow around that cycle lowers the cost without
    bound)."""
    sb = gen.grid_mincost_batch(batch=6, rows=rows, cols=cols, seed=seed)
    src, snk = sb.meta["source"], sb.meta["sink"]
    sb.lc[1] = 0.0
    sb.lc[1, src[1]], sb.lc[1, snk[1]] = 200.0, -200.0
    sb.uc[1] = sb.lc[1]
    t, h = sb.meta["tails"], sb.meta["heads"]
    a1 = 0
    a2 = int(np.nonzero((t == h[a1]) & (h == t[a1]))[0][0])
    sb.c[3, [a1, a2]] = -1.0
    sb.uv[3, [a1, a2]] = np.inf
    return sb


@pytest.mark.parametrize("rows,cols,threads", [(12, 12, 256), (24, 24, 512)])
def test_resident_matrix_batch_matches_oracle(pdhg, oracle_lib, rows, cols, threads):
    """Launches that keep the shared incidence matrix in registers (4 columns
    per thread for the 12x12 grid at 256 threads, 8 for the 24x24 grid at
    512): every instance ends as the oracle ends it (status and iteration
    count), with its objective or its certifying ray."""
    _say(f"case: {rows}x{cols} grid batch with certificates, {threads} threads (resident matrix)")
    sb = _grid_with_certificates(rows, cols, seed=3300 + rows)
    with pdhg.BatchSolver.from_shared(sb, threads=threads, iteration_limit=100000) as bs:
        x, y, res = bs.solve()
    for b in range(sb.batch):
        xo, yo, ro = oracle_lib.Oracle(sb.instance(b), iteration_limit=100000).solve()
        rb = res[b]
        _say(f"  instance {b}: {rb['status_name']} at {rb['iterations']} (oracle {ro['status_name']} at {ro['iterations']})")
        assert rb["status_name"] == ro["status_name"], (b, rb["status_name"], ro["status_name"])
        assert rb["iterations"] == ro["iterations"], (b, rb["iterations"], ro["iterations"])
        if ro["status_name"] == "primal_infeasible":
            assert b == 1 and rel_inf(to_np(y[b]), yo) <= 1e-8
        elif ro["status_name"] == "dual_infeasible":
            assert b == 3 and rel_inf(to_np(x[b]), xo) <= 1e-8
        else:
            assert ro["status_name"] == "optimal"
            assert _close(rb["primal_obj"], ro["primal_obj"])


@pytest.mark.parametrize("rows,cols,threads", [(12, 12, 256), (24, 24, 512)])
def test_resident_matrix_batch_without_ray_tests(pdhg, oracle_lib, rows, cols, threads):
    """The same launches with the infeasibility tests off (the leaner kernel):
    the feasible instances match the oracle's iteration counts and optima,
    the two without an optimum run to the iteration limit on both sides."""
    _say(f"case: {rows}x{cols} grid batch, ray tests off, {threads} threads (resident matrix)")
    sb = _grid_with_certificates(rows, cols, seed=3300 + rows)
    off = dict(iteration_limit=4000, eps_primal_infeasible=0.0, eps_dual_infeasible=0.0)
    with pdhg.BatchSolver.from_shared(sb, threads=threads, **off) as bs:
        x, y, res = bs.solve()
    for b in range(sb.batch):
        _, _, ro = oracle_lib.Oracle(sb.instance(b), **off).solve()
        rb = res[b]
        assert rb["status_name"] == ro["status_name"], (b, rb["status_name"], ro["status_name"])
        assert rb["iterations"] == ro["iterations"], (b, rb["iterations"], ro["iterations"])
        if b in (1, 3):
            assert rb["status_name"] == "iteration_limit"
        else:
            assert _close(rb["primal_obj"], ro["primal_obj"])
