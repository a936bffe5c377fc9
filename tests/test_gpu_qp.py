"""GPU parity of the rAPDHG (QP) path against the CPU oracle."""

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


def _dense_q(lp):
    q = gen.dense_from_csr(lp.n, lp.n, lp.q_rowptr, lp.q_colidx, lp.q_val)
    lp2 = gen.random_qp(lp.m, lp.n, seed=lp.meta["seed"])
    lp2.q_kind, lp2.q_dense = "dense", q
    return lp2


def _qp_cases():
    p = gen.portfolio_qp_batch(batch=2, n=120, seed=4600)
    yield "portfolio lowrank", gen.portfolio_instance(p, 0)
    qp = gen.random_qp(9, 14, seed=301)
    yield "random csr", qp
    yield "random dense", _dense_q(qp)


def test_qp_step_parity(pdhg, oracle_lib):
    for name, lp in _qp_cases():
        _say(f"case: QP step parity, {name}")
        orc = oracle_lib.Oracle(lp if lp.q_kind != "dense" else _as_csr(lp))
        sc = orc.scaling()
        with pdhg.Solver.from_lp(lp) as s:
            gs = s.scaling()
            assert abs(gs["norm_q"] - sc["norm_q"]) <= 1e-10 * max(sc["norm_q"], 1.0)
            rng = np.random.default_rng(1)
            x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
            xb, yb = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
            for k in (0, 3, 77):
                got = s.debug_qp_step(x, y, xb, yb, k, 1.7)
                ref = orc.qp_step(x, y, xb, yb, k, 1.7)
                for nm, g, r in zip(("x", "y", "xbar", "ybar"), got, ref):
                    assert rel_inf(to_np(g), r) <= 1e-12, (name, nm, k, rel_inf(to_np(g), r))


def _as_csr(lp):
    rp, ci, va = gen.csr_from_dense(lp.q_dense)
    q = gen.random_qp(lp.m, lp.n, seed=lp.meta["seed"])
    q.q_rowptr, q.q_colidx, q.q_val = rp, ci, va
    return q


def test_qp_solve_parity(pdhg, oracle_lib):
    for name, lp in _qp_cases():
        _say(f"case: QP solve parity, {name}")
        orc_lp = lp if lp.q_kind != "dense" else _as_csr(lp)
        xo, yo, ro = oracle_lib.Oracle(orc_lp).solve()
        with pdhg.Solver.from_lp(lp) as s:
            xg, yg, rg = s.solve()
        _say(f"  iterations gpu={rg['iterations']} oracle={ro['iterations']}")
        assert rg["status_name"] == "optimal" and rg["kkt_rel"] <= 1e-4
        assert abs(rg["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))
        kg = oracle_lib.kkt(orc_lp, to_np(xg), to_np(yg))
        assert abs(kg["kkt"] - rg["kkt_rel"]) <= 1e-9 + 1e-6 * kg["kkt"]


def test_qp_water_filling_on_gpu(pdhg):
    _say("case: QP water filling (F = 0)")
    p = gen.portfolio_qp_batch(batch=1, n=80, seed=4700)
    lp = gen.portfolio_instance(p, 0)
    lp.q_factor = np.zeros((lp.n, 1))
    with pdhg.Solver.from_lp(lp, eps=1e-9) as s:
        xg, yg, rg = s.solve()
    lo, hi = -10.0, 10.0
    for _ in range(200):
        lam = 0.5 * (lo + hi)
        tot = np.clip((lam - lp.c) / lp.q_diag, 0.0, 0.1).sum()
        lo, hi = (lam, hi) if tot < 1.0 else (lo, lam)
    ref = np.clip((0.5 * (lo + hi) - lp.c) / lp.q_diag, 0.0, 0.1)
    assert rg["status_name"] == "optimal"
    np.testing.assert_allclose(to_np(xg), ref, atol=1e-6)


@pytest.mark.parametrize("kind,m,n,seed,eps_d", [("duplicate_row", 40, 80, 0, 1e-8), ("boxed_sum", 20, 30, 1, 1e-8),
                                                 ("unbounded", 40, 80, 2, 1e-6), ("unbounded", 60, 120, 6, 1e-6)])
def test_qp_infeasibility_matches_oracle(pdhg, oracle_lib, kind, m, n, seed, eps_d):
    """rAPDHG: rays from the averages minus the anchor; the primal ray also
    needs Q dx = 0 (tested at 1e-6, where the test QPs certify in reach)."""
    _say(f"case: QP infeasibility detection, {kind} m={m} n={n} seed={seed}")
    lp = gen.infeasible_qp(kind, m, n, seed=seed)
    xo, yo, ro = oracle_lib.Oracle(lp, iteration_limit=100000, eps_dual_infeasible=eps_d).solve()
    with pdhg.Solver.from_lp(lp, iteration_limit=100000, eps_dual_infeasible=eps_d) as s:
        xg, yg, rg = s.solve()
    _say(f"  status gpu={rg['status_name']} oracle={ro['status_name']} "
         f"iterations gpu={rg['iterations']} oracle={ro['iterations']}")
    want = "dual_infeasible" if kind == "unbounded" else "primal_infeasible"
    assert ro["status_name"] == want and rg["status_name"] == want
    assert rg["iterations"] == ro["iterations"]
    ray_g, ray_o = (yg, yo) if want == "primal_infeasible" else (xg, xo)
    assert rel_inf(to_np(ray_g), ray_o) <= 1e-7
