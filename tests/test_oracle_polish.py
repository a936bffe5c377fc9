"""Pins of the oracle's feasibility polishing (Section 3: a post-processing
step that solves the feasibility-only problem from the current point; Appendix A:
eps_feas_polish = 1e-6, off by default) against what it promises, checked
outside the oracle: the polished primal point meets the constraints and the
polished dual point the dual constraints to 1e-6 relative (computed here with
numpy from the LP's data), its objective stays near HiGHS's optimum, and the
solve's status is unchanged."""

import numpy as np
import pytest

import gen
import oracle
from test_oracle_infeasibility import _dense


def _highs_value(lp):
    from test_oracle_heads import _exact
    return _exact(lp, lp.c)[1]


def _residuals(lp, x, y):
    """Relative primal residual |Ax - proj_[lc,uc](Ax)| / (1 + |b|) with x in
    its box, and relative dual residual of y: the part of c - A'y outside the
    cone the variable bounds allow, over 1 + |c|."""
    A = _dense(lp)
    ax = A @ x
    rp = ax - np.clip(ax, lp.lc, lp.uc)
    b = np.array([max(abs(l) if np.isfinite(l) else 0.0, abs(u) if np.isfinite(u) else 0.0)
                  for l, u in zip(lp.lc, lp.uc)])
    assert np.all(x >= lp.lv - 1e-12) and np.all(x <= lp.uv + 1e-12)
    g = lp.c - A.T @ y
    lo_f, up_f = np.isfinite(lp.lv), np.isfinite(lp.uv)
    # a reduced cost may be positive only at a finite lower bound and negative
    # only at a finite upper bound
    allowed = np.where(lo_f & up_f, g, np.where(lo_f, np.maximum(g, 0), np.where(up_f, np.minimum(g, 0), 0)))
    # y must have the sign its row allows: >= 0 needs a finite lower bound
    assert np.all(y[~np.isfinite(lp.lc)] <= 1e-12) and np.all(y[~np.isfinite(lp.uc)] >= -1e-12)
    return np.linalg.norm(rp) / (1 + np.linalg.norm(b)), np.linalg.norm(g - allowed) / (1 + np.linalg.norm(lp.c))


@pytest.mark.parametrize("make", [lambda: gen.planted_sparse_lp(200, 400, seed=11),
                                  lambda: gen.planted_sparse_lp(120, 300, seed=12),
                                  lambda: gen.tiny_boxed_lp(12, 20, seed=13),
                                  lambda: gen.grid_mincost_batch(batch=1, rows=6, cols=6, seed=14).instance(0)])
def test_polished_point_is_feasible_and_near_optimal(make):
    lp = make()
    x0, y0, r0 = oracle.Oracle(lp, eps=1e-4).solve()
    rp0, rd0 = _residuals(lp, x0, y0)
    x, y, r = oracle.Oracle(lp, eps=1e-4, feasibility_polishing=1).solve()
    assert r["status_name"] == "optimal"
    rp, rd = _residuals(lp, x, y)
    assert rp <= 1e-6 * (1 + 1e-9) and rd <= 1e-6 * (1 + 1e-9), (rp, rd, rp0, rd0)
    # the reported terms are those of the polished point
    assert abs(r["rel_primal"] - rp) <= 1e-12 + 1e-9 * rp and abs(r["rel_dual"] - rd) <= 1e-12 + 1e-9 * rd
    if max(rp0, rd0) > 1e-6:
        assert r["polish_iterations"] > 0
    assert r["iterations"] == r0["iterations"] + r["polish_iterations"]
    # started near an optimum, polishing stays near one
    v = _highs_value(lp)
    assert abs(np.dot(lp.c, x) - v) <= 1e-2 * (1 + abs(v)), (np.dot(lp.c, x), v)


def test_polishing_is_off_by_default_and_skips_non_optimal_ends():
    lp = gen.planted_sparse_lp(80, 160, seed=15)
    r = oracle.Oracle(lp).solve()[2]
    assert r["polish_iterations"] == 0
    r = oracle.Oracle(lp, iteration_limit=50, feasibility_polishing=1).solve()[2]
    assert r["status_name"] == "iteration_limit" and r["polish_iterations"] == 0
