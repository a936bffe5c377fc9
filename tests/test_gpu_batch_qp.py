"""GPU parity of the batched rAPDHG path (portfolio QPs, Q_b = F F' + diag(d_b)
with F shared) against the CPU oracle: full solves, the unrolled forward with
its frozen schedule, and the reverse pass (gradients in c, l_c, u_c and d)."""

import sys
from types import SimpleNamespace

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


def _batch(p):
    B = p["c"].shape[0]
    return SimpleNamespace(m=p["m"], n=p["n"], rowptr=p["rowptr"], colidx=p["colidx"], val=p["val"],
                           c=p["c"], lc=np.tile(p["lc"], (B, 1)), uc=np.tile(p["uc"], (B, 1)),
                           lv=np.tile(p["lv"], (B, 1)), uv=np.tile(p["uv"], (B, 1)),
                           q_factor=p["F"], q_diag=p["d"])


def test_batch_qp_solve_matches_oracle(pdhg, oracle_lib):
    _say("case: batched rAPDHG solve, 6 portfolio QPs n=90 rank 6, eps 1e-6")
    p = gen.portfolio_qp_batch(batch=6, n=90, rank=6, seed=4700)
    with pdhg.BatchSolver.from_shared(_batch(p), eps=1e-6) as bs:
        x, y, res = bs.solve()
        for b in range(6):
            lp = gen.portfolio_instance(p, b)
            xo, yo, ro = oracle_lib.Oracle(lp, eps=1e-6).solve()
            r = res[b]
            assert r["status"] == 1 and ro["status"] == 1, (b, r, ro)
            assert r["kkt_rel"] <= 1e-6
            assert abs(r["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))
            # same algorithm and check period: the counts agree up to one period
            assert abs(r["iterations"] - ro["iterations"]) <= 64, (b, r["iterations"], ro["iterations"])
            assert rel_inf(to_np(x[b]), xo) <= 1e-4
            kk = oracle_lib.kkt(lp, to_np(x[b]), to_np(y[b]))
            assert kk["kkt"] <= 2e-6


@pytest.mark.parametrize("T", [173, 200])
def test_batch_qp_unrolled_and_adjoint_match_oracle(pdhg, oracle_lib, T):
    _say(f"case: batched unrolled rAPDHG + adjoint, 4 portfolio QPs n=70 rank 4, T={T}")
    p = gen.portfolio_qp_batch(batch=4, n=70, rank=4, seed=4800)
    rng = np.random.default_rng(T)
    with pdhg.BatchSolver.from_shared(_batch(p)) as bs:
        x, y = bs.unrolled(T)
        gx = rng.standard_normal((4, 70))
        gy = rng.standard_normal((4, 1))
        gc, glc, guc, gd = bs.backward(gx, gy)
        for b in range(4):
            o = oracle_lib.Oracle(gen.portfolio_instance(p, b))
            xo, yo, sr, sw = o.unrolled_qp(T)
            assert rel_inf(to_np(x[b]), xo) <= 1e-10, (b, rel_inf(to_np(x[b]), xo))
            assert rel_inf(to_np(y[b]), yo) <= 1e-10
            gco, glco, guco, gdo = o.backward_qp(T, sr, sw, gx[b], gy[b])
            assert rel_inf(to_np(gc[b]), gco) <= 1e-9, (b, rel_inf(to_np(gc[b]), gco))
            assert rel_inf(to_np(glc[b]), glco) <= 1e-9
            assert rel_inf(to_np(guc[b]), guco) <= 1e-9
            assert rel_inf(to_np(gd[b]), gdo) <= 1e-9, (b, rel_inf(to_np(gd[b]), gdo))


def test_batch_qp_rejects_bad_input(pdhg):
    _say("case: batched QP argument errors")
    p = gen.portfolio_qp_batch(batch=2, n=40, rank=33, seed=4900)
    with pytest.raises(Exception):
        pdhg.BatchSolver.from_shared(_batch(p))
    p = gen.portfolio_qp_batch(batch=2, n=40, rank=3, seed=4901)
    p["F"] = p["F"].copy()
    p["F"][5, 1] = np.nan
    with pytest.raises(Exception):
        pdhg.BatchSolver.from_shared(_batch(p))
