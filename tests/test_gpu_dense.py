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
