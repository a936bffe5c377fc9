"""GPU parity of the dense-matrix path (row-major A) against the CPU oracle."""

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


def _step(pdhg, oracle_lib, lp, compare_eta=True, ks=(0, 9)):
    orc = oracle_lib.Oracle(lp) if compare_eta else oracle_lib.Oracle(lp, power_max_iters=1)
    sc = orc.scaling()
    with pdhg.Solver.from_lp(lp) as s:
        gs = s.scaling()
        assert rel_inf(to_np(gs["dc"]), sc["dc"]) <= 1e-12
        assert rel_inf(to_np(gs["dr"]), sc["dr"]) <= 1e-12
        if compare_eta:
            assert abs(gs["eta"] - sc["eta"]) <= 1e-10 * sc["eta"]
        rng = np.random.default_rng(3)
        x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
        x0, y0 = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
        tau, sigma = sc["eta"] / sc["omega"], sc["eta"] * sc["omega"]
        for k in ks:
            got = s.debug_step(x, y, x0, y0, k, tau, sigma)
            ref = orc.lp_step(x, y, x0, y0, k, tau, sigma)
            for nm, g, r in zip(("xhat", "yhat", "xnew", "ynew"), got, ref):
                assert rel_inf(to_np(g), r) <= 1e-12, (nm, k, rel_inf(to_np(g), r))


def test_dense_small_step_and_solve(pdhg, oracle_lib):
    _say("case: dense planted LP 150 x 300, step and solve parity")
    lp = gen.dense_planted_lp(150, 300, seed=2001)
    _step(pdhg, oracle_lib, lp)
    xo, yo, ro = oracle_lib.Oracle(lp).solve()
    with pdhg.Solver.from_lp(lp) as s:
        xg, yg, rg = s.solve()
    _say(f"  iterations gpu={rg['iterations']} oracle={ro['iterations']}")
    assert rg["status_name"] == "optimal" and rg["kkt_rel"] <= 1e-4
    assert abs(rg["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))


def test_dense_knapsack_shape_step_and_solve(pdhg, oracle_lib):
    """Few long rows, as in the knapsack shape: a workgroup per four rows with
    every lane through the unrolled loads (20,000 columns), one row split in
    the column pass; step and solve against the oracle."""
    _say("case: dense knapsack-shaped LP 30 x 20000, step and solve parity")
    lp = gen.dense_knapsack_lp(d=30, items=20000, seed=2501)
    _step(pdhg, oracle_lib, lp)
    xo, yo, ro = oracle_lib.Oracle(lp).solve()
    with pdhg.Solver.from_lp(lp) as s:
        xg, yg, rg = s.solve()
    _say(f"  iterations gpu={rg['iterations']} oracle={ro['iterations']}")
    assert ro["status_name"] == "optimal" and rg["status_name"] == "optimal" and rg["kkt_rel"] <= 1e-4
    assert abs(rg["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))


def test_dense_matches_csr_path(pdhg):
    _say("case: dense and CSR storage of the same LP give the same solve")
    lp = gen.dense_planted_lp(120, 260, seed=2002)
    rp, ci, va = gen.csr_from_dense(lp.dense)
    sp = gen.LP(lp.m, lp.n, rp, ci, va, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    with pdhg.Solver.from_lp(lp) as s:
        _, _, rd = s.solve()
    with pdhg.Solver.from_lp(sp) as s:
        _, _, rs = s.solve()
    assert abs(rd["primal_obj"] - rs["primal_obj"]) <= 1e-6 * (1 + abs(rs["primal_obj"]))


@pytest.mark.timeout(900)
def test_dense_step_parity_large(pdhg, oracle_lib):
    """Full-size dense LP (20,000 x 40,000): scaling and one iteration."""
    _say("case: dense step parity at full size 20000 x 40000 (generation + oracle take minutes)")
    lp = gen.dense_planted_lp(seed=2000)
    _say("  generated")
    _step(pdhg, oracle_lib, lp, compare_eta=False, ks=(4,))


def _dense_copy(lp):
    import copy
    d = copy.copy(lp)
    d.dense = gen.dense_from_csr(lp.m, lp.n, lp.rowptr, lp.colidx, lp.val)
    d.rowptr = d.colidx = d.val = None
    return d


@pytest.mark.parametrize("kind,m,n,seed", [("duplicate_row", 60, 120, 0), ("boxed_sum", 30, 50, 3),
                                           ("unbounded", 400, 800, 1), ("duplicate_row", 1100, 2200, 4)])
def test_dense_infeasibility_certificates_match_oracle(pdhg, oracle_lib, kind, m, n, seed):
    """Row-major storage: the dense check kernels produce the same ray terms
    (a workgroup per row below 1,024 rows, four rows per wave above)."""
    _say(f"case: dense infeasibility detection, {kind} m={m} n={n} seed={seed}")
    lp = _dense_copy(gen.infeasible_lp(kind, m, n, seed=seed))
    xo, yo, ro = oracle_lib.Oracle(lp, iteration_limit=100000).solve()
    with pdhg.Solver.from_lp(lp, iteration_limit=100000) as s:
        xg, yg, rg = s.solve()
    _say(f"  status gpu={rg['status_name']} oracle={ro['status_name']} "
         f"iterations gpu={rg['iterations']} oracle={ro['iterations']}")
    want = "dual_infeasible" if kind == "unbounded" else "primal_infeasible"
    assert ro["status_name"] == want and rg["status_name"] == want
    assert rg["iterations"] == ro["iterations"]
    if want == "primal_infeasible":
        assert rel_inf(to_np(yg), yo) <= 1e-8
    else:
        assert rel_inf(to_np(xg), xo) <= 1e-8


def test_dense_kernel_timing(pdhg):
    _say("case: dense planted LP 150 x 300, HIP-event timing of one check period")
    lp = gen.dense_planted_lp(150, 300, seed=2001)
    with pdhg.Solver.from_lp(lp, timing_chunk=1) as s:
        _, _, r = s.solve()
    assert r["status_name"] == "optimal"
    assert r["kernel_samples"] > 0
    assert r["kernel_primal_ms"] > 0 and r["kernel_dual_ms"] > 0
