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


def _with_group_limits(p, groups=40, size=5, cap=0.3, seed=0):
    """The portfolio plus `groups` rows sum_{j in S} x_j <= cap over random
    asset groups S: many short rows, so the per-thread row path runs."""
    rng = np.random.default_rng(seed)
    n = p["n"]
    rows = [np.arange(n)] + [np.sort(rng.choice(n, size=size, replace=False)) for _ in range(groups)]
    rowptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    q = dict(p)
    q.update(m=1 + groups, rowptr=rowptr, colidx=np.concatenate(rows).astype(np.int32),
             val=np.ones(rowptr[-1]), lc=np.r_[1.0, np.full(groups, -np.inf)],
             uc=np.r_[1.0, np.full(groups, cap)])
    return q


def _instance(p, b):
    lp = gen.portfolio_instance(p, b)
    lp.m, lp.rowptr, lp.colidx, lp.val = p["m"], p["rowptr"], p["colidx"], p["val"]
    lp.lc, lp.uc = p["lc"].copy(), p["uc"].copy()
    return lp


@pytest.mark.parametrize("rows", ["budget", "groups"])
def test_batch_qp_rows_paths_match_oracle(pdhg, oracle_lib, rows):
    _say(f"case: batched rAPDHG unrolled + adjoint, constraint rows '{rows}'")
    p = gen.portfolio_qp_batch(batch=3, n=60, rank=3, seed=4750)
    if rows == "groups":
        p = _with_group_limits(p)
    T = 160
    rng = np.random.default_rng(5)
    with pdhg.BatchSolver.from_shared(_batch(p)) as bs:
        x, y = bs.unrolled(T)
        gx = rng.standard_normal((3, p["n"]))
        gy = rng.standard_normal((3, p["m"]))
        gc, glc, guc, gd = bs.backward(gx, gy)
        xs, ys, res = bs.solve()
        for b in range(3):
            o = oracle_lib.Oracle(_instance(p, b))
            xo, yo, sr, sw = o.unrolled_qp(T)
            assert rel_inf(to_np(x[b]), xo) <= 1e-10
            assert rel_inf(to_np(y[b]), yo) <= 1e-10
            gco, glco, guco, gdo = o.backward_qp(T, sr, sw, gx[b], gy[b])
            assert rel_inf(to_np(gc[b]), gco) <= 1e-9
            assert rel_inf(to_np(glc[b]), glco) <= 1e-9
            assert rel_inf(to_np(guc[b]), guco) <= 1e-9
            assert rel_inf(to_np(gd[b]), gdo) <= 1e-9
            xso, yso, ro = o.solve()
            assert res[b]["status"] == 1 and ro["status"] == 1
            assert abs(res[b]["iterations"] - ro["iterations"]) <= 64
            assert abs(res[b]["primal_obj"] - ro["primal_obj"]) <= 1e-5 * (1 + abs(ro["primal_obj"]))


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
