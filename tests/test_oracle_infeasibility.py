"""Pins of the oracle's infeasibility certificates (Section 3 names the
detection; Appendix A its 1e-8 tolerances) against facts outside it:
HiGHS's status for the same LP, the returned rays checked by other means
(a dual ray by maximising y'Ax over the variable box, a primal ray by its
definition as a direction of unbounded descent), and no certificate on
feasible LPs."""

import numpy as np
import pytest

import gen
import oracle
from test_oracle_heads import _exact


def _highs_status(lp):
    from scipy.optimize import linprog
    import scipy.sparse as sp
    A = sp.csr_matrix((lp.val, lp.colidx, lp.rowptr), shape=(lp.m, lp.n))
    eq = np.isfinite(lp.lc) & np.isfinite(lp.uc) & (lp.lc == lp.uc)
    ub, rhs = [], []
    for i in np.where(~eq)[0]:
        if np.isfinite(lp.uc[i]):
            ub.append(A[i]); rhs.append(lp.uc[i])
        if np.isfinite(lp.lc[i]):
            ub.append(-A[i]); rhs.append(-lp.lc[i])
    kw = dict(A_eq=A[eq], b_eq=lp.lc[eq]) if eq.any() else {}
    if ub:
        kw.update(A_ub=sp.vstack(ub), b_ub=np.array(rhs))
    bounds = [(None if not np.isfinite(l) else l, None if not np.isfinite(u) else u)
              for l, u in zip(lp.lv, lp.uv)]
    return linprog(lp.c, bounds=bounds, method="highs", **kw).status   # 2 infeasible, 3 unbounded


def _dense(lp):
    return gen.dense_from_csr(lp.m, lp.n, lp.rowptr, lp.colidx, lp.val)


@pytest.mark.parametrize("kind,m,n,seed", [("duplicate_row", 60, 120, 0), ("duplicate_row", 400, 800, 1),
                                           ("boxed_sum", 8, 12, 2), ("boxed_sum", 30, 50, 3)])
def test_primal_infeasible_certificate(kind, m, n, seed):
    lp = gen.infeasible_lp(kind, m, n, seed=seed)
    assert _highs_status(lp) == 2
    x, y, r = oracle.Oracle(lp, iteration_limit=100000).solve()
    assert r["status_name"] == "primal_infeasible", r
    if kind == "boxed_sum":
        # equality rows A x = b, x in [0, 1]^n: every feasible x has y'Ax = y'b,
        # but over the box y'Ax is at most sum_j max(0, (A'y)_j) < y'b
        g = _dense(lp).T @ y
        assert np.sum(np.maximum(g, 0.0)) < np.dot(lp.lc, y) - 0.5
    else:
        # Farkas: every feasible x has y_i (Ax)_i >= y_i l_i where y_i > 0 (a
        # finite lower bound) and >= y_i u_i where y_i < 0 (a finite upper
        # bound), so y'Ax >= b(y); over x >= 0, y'Ax <= 0 once A'y <= 0.
        # The ray is scaled to b(y) = 1 and holds these up to 1e-8.
        ge = np.isfinite(lp.lc) & ~np.isfinite(lp.uc)
        le = ~np.isfinite(lp.lc) & np.isfinite(lp.uc)
        assert np.min(y[ge], initial=0.0) >= -1e-8 and np.max(y[le], initial=0.0) <= 1e-8
        pos, neg = (y > 0) & np.isfinite(lp.lc), (y < 0) & np.isfinite(lp.uc)
        b_y = np.dot(lp.lc[pos], y[pos]) + np.dot(lp.uc[neg], y[neg])
        assert abs(b_y - 1.0) <= 1e-9
        assert np.max(_dense(lp).T @ y) <= 1e-8 * (1 + 1e-9)


@pytest.mark.parametrize("m,n,seed", [(60, 120, 0), (60, 120, 2), (400, 800, 1)])
def test_dual_infeasible_certificate(m, n, seed):
    lp = gen.infeasible_lp("unbounded", m, n, seed=seed)
    assert _highs_status(lp) == 3
    x, y, r = oracle.Oracle(lp, iteration_limit=100000).solve()
    assert r["status_name"] == "dual_infeasible", r
    d = x
    ad = _dense(lp) @ d
    eq = lp.lc == lp.uc
    assert abs(np.dot(lp.c, d) + 1.0) <= 1e-12      # normalised descent
    assert np.max(np.abs(ad[eq])) <= 1e-8            # stays on the equality rows
    assert np.min(ad[~eq & np.isfinite(lp.lc)], initial=0.0) >= -1e-8   # >= rows: A d >= 0
    assert np.max(ad[~eq & np.isfinite(lp.uc)], initial=0.0) <= 1e-8    # <= rows: A d <= 0
    assert np.min(d) >= -1e-8                        # x >= 0
    # the planted direction moves A x off the one-sided rows' bounds
    assert d[-1] > 0.0 and np.max(np.abs(ad[~eq])) > 1e-3


def test_no_certificate_on_feasible_lps_and_switches():
    for seed in range(4):
        lp = gen.planted_sparse_lp(80, 160, seed=7000 + seed)
        assert oracle.Oracle(lp, iteration_limit=100000).solve()[2]["status_name"] == "optimal"
    lp = gen.infeasible_lp("duplicate_row", 60, 120, seed=0)
    r = oracle.Oracle(lp, eps_primal_infeasible=0.0, iteration_limit=3000).solve()[2]
    assert r["status_name"] == "iteration_limit"
    lp = gen.infeasible_lp("unbounded", 60, 120, seed=0)
    r = oracle.Oracle(lp, eps_dual_infeasible=0.0, iteration_limit=3000).solve()[2]
    assert r["status_name"] == "iteration_limit"


def test_no_rows_unbounded_and_boxed():
    """No constraint rows: with x >= 0 and one negative cost the objective is
    unbounded along that coordinate alone (the ray is e_7 with c'd = -1);
    with a box on every variable the same LP has an optimum."""
    n = 40
    c = np.random.default_rng(0).uniform(0.5, 2.0, n)
    c[7] = -1.0
    lp = gen.LP(0, n, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), c, np.zeros(0), np.zeros(0),
                np.zeros(n), np.full(n, np.inf))
    x, y, r = oracle.Oracle(lp, iteration_limit=100000).solve()
    assert r["status_name"] == "dual_infeasible"
    e = np.zeros(n); e[7] = 1.0
    np.testing.assert_allclose(x, e, atol=1e-12)
    lp.uv = np.full(n, 5.0)
    x, y, r = oracle.Oracle(lp, iteration_limit=100000).solve()
    assert r["status_name"] == "optimal" and abs(x[7] - 5.0) <= 1e-9


def _dense_q(lp):
    return gen.dense_from_csr(lp.n, lp.n, lp.q_rowptr, lp.q_colidx, lp.q_val)


@pytest.mark.parametrize("kind,m,n,seed", [("duplicate_row", 40, 80, 0), ("boxed_sum", 20, 30, 1)])
def test_qp_primal_infeasible_certificate(kind, m, n, seed):
    """A QP is infeasible exactly when its constraints are: HiGHS's status of
    the constraint set and the Farkas ray checks of the LP tests."""
    lp = gen.infeasible_qp(kind, m, n, seed=seed)
    assert _highs_status(lp) == 2
    x, y, r = oracle.Oracle(lp, iteration_limit=100000).solve()
    assert r["status_name"] == "primal_infeasible", r
    if kind == "boxed_sum":
        g = _dense(lp).T @ y
        assert np.sum(np.maximum(g, 0.0)) < np.dot(lp.lc, y) - 0.5
    else:
        pos, neg = (y > 0) & np.isfinite(lp.lc), (y < 0) & np.isfinite(lp.uc)
        assert abs(np.dot(lp.lc[pos], y[pos]) + np.dot(lp.uc[neg], y[neg]) - 1.0) <= 1e-9
        assert np.max(_dense(lp).T @ y) <= 1e-8 * (1 + 1e-9)


@pytest.mark.parametrize("m,n,seed", [(40, 80, 2), (60, 120, 6)])
def test_qp_dual_infeasible_certificate(m, n, seed):
    """Unbounded QP (the added column has no Q entries): the primal ray has
    c'd = -1, Q d = 0, A d in the rows' recession cones and d >= 0, checked
    with the dense Q and A. The ray's Q term converges more slowly than an
    LP's, so this test uses eps_dual_infeasible = 1e-6."""
    lp = gen.infeasible_qp("unbounded", m, n, seed=seed)
    x, y, r = oracle.Oracle(lp, iteration_limit=100000, eps_dual_infeasible=1e-6).solve()
    assert r["status_name"] == "dual_infeasible", r
    d = x
    assert abs(np.dot(lp.c, d) + 1.0) <= 1e-12
    assert np.max(np.abs(_dense_q(lp) @ d)) <= 1e-6
    ad = _dense(lp) @ d
    eq = lp.lc == lp.uc
    assert np.max(np.abs(ad[eq])) <= 1e-6
    assert np.min(ad[~eq & np.isfinite(lp.lc)], initial=0.0) >= -1e-6
    assert np.max(ad[~eq & np.isfinite(lp.uc)], initial=0.0) <= 1e-6
    assert np.min(d) >= -1e-6 and d[-1] > 0.0


_KINDS = ["optimal", "primal_infeasible", "dual_infeasible", "optimal", "dual_infeasible", "primal_infeasible"]


@pytest.mark.parametrize("m,n,r,seed", [(40, 80, 4, 0), (60, 120, 6, 1)])
def test_lowrank_qp_batch_certificates(m, n, r, seed):
    """The shared-A QP batch with Q_b = F F' + diag(d_b): each instance ends
    as it was built, checked by means outside the oracle: HiGHS's status of
    the constraint set (c = 0), the Farkas checks of the dual rays, and the
    primal rays' definition (c'd = -1, Q d = 0, A d in the rows' recession
    cones, d >= 0) with the dense Q and A, at the default 1e-8 tolerances."""
    import copy
    sb = gen.mixed_qp_batch(_KINDS, m, n, r, seed)
    a = gen.dense_from_csr(sb.m, sb.n, sb.rowptr, sb.colidx, sb.val)
    for b, kind in enumerate(_KINDS):
        lp = sb.instance(b)
        feas = copy.copy(lp)
        feas.c = np.zeros(lp.n)
        assert _highs_status(feas) == (2 if kind == "primal_infeasible" else 0), (b, kind)
        x, y, res = oracle.Oracle(lp, iteration_limit=100000).solve()
        assert res["status_name"] == kind, (b, kind, res)
        if kind == "primal_infeasible":
            ge = np.isfinite(lp.lc) & ~np.isfinite(lp.uc)
            le = ~np.isfinite(lp.lc) & np.isfinite(lp.uc)
            assert np.min(y[ge], initial=0.0) >= -1e-8 and np.max(y[le], initial=0.0) <= 1e-8
            pos, neg = (y > 0) & np.isfinite(lp.lc), (y < 0) & np.isfinite(lp.uc)
            assert abs(np.dot(lp.lc[pos], y[pos]) + np.dot(lp.uc[neg], y[neg]) - 1.0) <= 1e-9
            assert np.max(a.T @ y) <= 1e-8 * (1 + 1e-9)
        elif kind == "dual_infeasible":
            d = x
            q = sb.q_factor @ sb.q_factor.T + np.diag(sb.q_diag[b])
            assert abs(np.dot(lp.c, d) + 1.0) <= 1e-12
            assert np.max(np.abs(q @ d)) <= 1e-8 * (1 + 1e-6)
            ad = a @ d
            eq = lp.lc == lp.uc
            assert np.max(np.abs(ad[eq])) <= 1e-8 * (1 + 1e-6)
            assert np.min(ad[~eq & np.isfinite(lp.lc)], initial=0.0) >= -1e-8 * (1 + 1e-6)
            assert np.max(ad[~eq & np.isfinite(lp.uc)], initial=0.0) <= 1e-8 * (1 + 1e-6)
            assert np.min(d) >= -1e-8 and d[-1] > 0.0
