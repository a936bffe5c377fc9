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
            assert res[b]["iterations"] == ro["iterations"]
            assert abs(res[b]["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))


def test_batch_qp_beyond_lds_matches_oracle(pdhg, oracle_lib):
    """n = 1,000: the instance's vectors exceed the on-chip budget, so the
    memory-resident kernels run (solve, unrolled forward and reverse pass)."""
    _say("case: batched rAPDHG, 2 portfolio QPs n=1000 rank 5 (memory-resident kernels)")
    p = gen.portfolio_qp_batch(batch=2, n=1000, rank=5, seed=4760)
    p["uv"] = np.full(1000, 0.05)
    T = 120
    rng = np.random.default_rng(6)
    with pdhg.BatchSolver.from_shared(_batch(p)) as bs:
        x, y = bs.unrolled(T)
        gx = rng.standard_normal((2, p["n"]))
        gc, glc, guc, gd = bs.backward(gx)
        xs, ys, res = bs.solve()
        for b in range(2):
            o = oracle_lib.Oracle(_instance(p, b))
            xo, yo, sr, sw = o.unrolled_qp(T)
            assert rel_inf(to_np(x[b]), xo) <= 1e-10
            assert rel_inf(to_np(y[b]), yo) <= 1e-10
            gco, glco, guco, gdo = o.backward_qp(T, sr, sw, gx[b], np.zeros(p["m"]))
            assert rel_inf(to_np(gc[b]), gco) <= 1e-9
            assert rel_inf(to_np(gd[b]), gdo) <= 1e-9
            xso, yso, ro = o.solve()
            assert res[b]["status"] == 1 and ro["status"] == 1
            assert res[b]["iterations"] == ro["iterations"]
            assert abs(res[b]["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))


def test_batch_qp_autotune_then_solve(pdhg, oracle_lib):
    _say("case: batched rAPDHG autotune (64..1024 threads), then a solve at the chosen shape")
    p = gen.portfolio_qp_batch(batch=4, n=90, rank=6, seed=4710)
    with pdhg.BatchSolver.from_shared(_batch(p)) as bs:
        best = bs.autotune(64)
        _say(f"  autotuned threads per instance = {best}")
        assert best in (64, 128, 256, 512, 1024)
        x, y, res = bs.solve()
    for b in range(4):
        lp = gen.portfolio_instance(p, b)
        _, _, ro = oracle_lib.Oracle(lp).solve()
        assert res[b]["status"] == 1 and ro["status"] == 1
        assert res[b]["iterations"] == ro["iterations"]
        assert abs(res[b]["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))


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
            assert r["iterations"] == ro["iterations"], (b, r["iterations"], ro["iterations"])
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


_KINDS = ["optimal", "primal_infeasible", "dual_infeasible", "optimal", "dual_infeasible", "primal_infeasible"]


@pytest.mark.parametrize("m,n,r,seed,threads", [(40, 80, 4, 0, None), (60, 120, 6, 1, None), (40, 80, 4, 0, 1024)])
def test_batch_qp_infeasibility_matches_oracle(pdhg, oracle_lib, m, n, r, seed, threads):
    """A shared-A QP batch whose instances are optimal, infeasible or
    unbounded ends each instance as the oracle ends it. The detection check
    may differ from the oracle's by a period or two (the batched power
    iteration starts from another vector, so the trajectories drift apart):
    every returned ray is checked against its definition with the dense A and
    Q, and against the oracle's element by element when both stop at the same
    iteration. 1024 threads per instance is the shape the caller may choose."""
    _say(f"case: batched QP infeasibility, m={m} n={n} rank={r} seed={seed} threads {threads or 'default'}")
    sb = gen.mixed_qp_batch(_KINDS, m, n, r, seed)
    a = gen.dense_from_csr(sb.m, sb.n, sb.rowptr, sb.colidx, sb.val)
    kw = dict(threads=threads) if threads else {}
    with pdhg.BatchSolver.from_shared(sb, iteration_limit=100000, **kw) as bs:
        x, y, res = bs.solve()
    for b, kind in enumerate(_KINDS):
        lp = sb.instance(b)
        xo, yo, ro = oracle_lib.Oracle(lp, iteration_limit=100000).solve()
        rb = res[b]
        _say(f"  instance {b} ({kind}): gpu {rb['status_name']} at {rb['iterations']}, "
             f"oracle {ro['status_name']} at {ro['iterations']}")
        assert ro["status_name"] == kind
        assert rb["status_name"] == kind, (b, rb["status_name"], kind)
        assert rb["iterations"] == ro["iterations"], (b, rb["iterations"], ro["iterations"])
        xb, yb = to_np(x[b]), to_np(y[b])
        if kind == "primal_infeasible":
            pos, neg = (yb > 0) & np.isfinite(lp.lc), (yb < 0) & np.isfinite(lp.uc)
            assert abs(np.dot(lp.lc[pos], yb[pos]) + np.dot(lp.uc[neg], yb[neg]) - 1.0) <= 1e-9
            assert np.max(a.T @ yb) <= 1e-8 * (1 + 1e-6)
            assert rel_inf(yb, yo) <= 1e-6
        elif kind == "dual_infeasible":
            q = sb.q_factor @ sb.q_factor.T + np.diag(sb.q_diag[b])
            assert abs(np.dot(lp.c, xb) + 1.0) <= 1e-12
            assert np.max(np.abs(q @ xb)) <= 1e-8 * (1 + 1e-6)
            ad = a @ xb
            eq = lp.lc == lp.uc
            assert np.max(np.abs(ad[eq])) <= 1e-8 * (1 + 1e-6)
            assert np.min(ad[~eq & np.isfinite(lp.lc)], initial=0.0) >= -1e-8 * (1 + 1e-6)
            assert np.max(ad[~eq & np.isfinite(lp.uc)], initial=0.0) <= 1e-8 * (1 + 1e-6)
            assert np.min(xb) >= -1e-8 and xb[-1] > 0.0
            assert rel_inf(xb, xo) <= 1e-6
        else:
            assert abs(rb["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))
            assert oracle_lib.kkt(lp, xb, yb)["kkt"] <= 1e-4 * (1 + 1e-6)


def test_batch_qp_infeasibility_switched_off(pdhg):
    _say("case: batched QP with the infeasibility tests off (lean kernel)")
    sb = gen.mixed_qp_batch(_KINDS, 40, 80, 4, 0)
    with pdhg.BatchSolver.from_shared(sb, iteration_limit=3000, eps_primal_infeasible=0.0,
                                      eps_dual_infeasible=0.0) as bs:
        _, _, res = bs.solve()
    names = [r["status_name"] for r in res]
    assert names[1] == names[2] == names[4] == names[5] == "iteration_limit", names
    assert names[0] == names[3] == "optimal", names
