"""Pins for the CPU oracle: each test checks it against something other than
itself (textbook projections, planted optimal pairs, HiGHS, vertex
enumeration, Dijkstra, water-filling, explicit dense matrices, finite
differences)."""

import itertools

import numpy as np
import pytest

import gen

INF = np.inf


def _orc(lp, **kw):
    import oracle
    return oracle.Oracle(lp, **kw)


def _dense_scaled(lp, sc):
    return sc["dr"][:, None] * lp.to_dense() * sc["dc"][None, :]


# ---------------------------------------------------------------------------
# one iteration


def test_step_linear_special_case(oracle_lib):
    """No variable bounds, all rows equalities: the PDHG step of eq. (pdhg-lp)
    is linear, xhat = x - tau (c - A'y), yhat = y - sigma (A(2xhat - x) - b)."""
    lp = gen.planted_sparse_lp(30, 50, density=0.2, seed=11)
    lp.lv[:] = -INF
    lp.uv[:] = INF
    b = lp.matvec(np.random.default_rng(1).random(lp.n))
    lp.lc, lp.uc = b.copy(), b.copy()
    o = _orc(lp, ruiz_iters=0, pock_chambolle=0)   # A~ = A, no scaling
    a = lp.to_dense()
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    tau, sigma = 0.3, 0.7
    xh, yh, _, _ = o.lp_step(x, y, x, y, 0, tau, sigma)
    xr = x - tau * (lp.c - a.T @ y)
    yr = y - sigma * (a @ (2 * xr - x) - b)
    np.testing.assert_allclose(xh, xr, rtol=0, atol=1e-12 * np.abs(xr).max())
    np.testing.assert_allclose(yh, yr, rtol=0, atol=1e-12 * np.abs(yr).max())


def _prox_piecewise(w, sigma, l, u):
    """argmin_y p(y) + |y - w|^2/(2 sigma), p(y) = u y^- - l y^+, solved per
    case: y = w + sigma l if that is > 0, y = w + sigma u if that is < 0,
    else 0."""
    out = np.zeros_like(w)
    for i in range(len(w)):
        if np.isfinite(l[i]) and w[i] + sigma * l[i] > 0:
            out[i] = w[i] + sigma * l[i]
        elif np.isfinite(u[i]) and w[i] + sigma * u[i] < 0:
            out[i] = w[i] + sigma * u[i]
    return out


def test_step_projections_textbook(oracle_lib):
    """Box clamp for x and the piecewise minimiser of the dual prox for y,
    on a problem with every kind of bound (eq. (pdhg-lp), Section 2 cones)."""
    lp = gen.tiny_boxed_lp(8, 12, seed=5)
    lp.lv[::3] = -INF
    lp.uv[1::4] = INF
    o = _orc(lp, ruiz_iters=0, pock_chambolle=0)
    a = lp.to_dense()
    rng = np.random.default_rng(3)
    for trial in range(5):
        x, y = rng.standard_normal(lp.n) * 2, rng.standard_normal(lp.m) * 2
        tau, sigma = rng.uniform(0.1, 1.0, 2)
        xh, yh, _, _ = o.lp_step(x, y, x, y, 0, tau, sigma)
        xr = np.clip(x - tau * (lp.c - a.T @ y), lp.lv, lp.uv)
        w = y - sigma * (a @ (2 * xr - x))
        yr = _prox_piecewise(w, sigma, lp.lc, lp.uc)
        np.testing.assert_allclose(xh, xr, rtol=0, atol=1e-12)
        np.testing.assert_allclose(yh, yr, rtol=0, atol=1e-12)
        # yhat lies in Y exactly (sign constraints of Section 2)
        assert np.all(yh[~np.isfinite(lp.lc)] <= 0.0)
        assert np.all(yh[~np.isfinite(lp.uc)] >= 0.0)


def test_planted_pair_is_fixed_point(oracle_lib):
    """A planted optimal pair is a fixed point of one r2HPDHG iteration, and
    Halpern from the anchor z* stays at z* (Algorithm 1)."""
    lp = gen.planted_sparse_lp(seed=0)
    o = _orc(lp)
    sc = o.scaling()
    xs, ys = lp.x_star / sc["dc"], lp.y_star / sc["dr"]
    for tau, sigma, k in ((sc["eta"] / sc["omega"], sc["eta"] * sc["omega"], 0), (0.05, 3.0, 17)):
        xh, yh, xn, yn = o.lp_step(xs, ys, xs, ys, k, tau, sigma)
        for got, ref in ((xh, xs), (yh, ys), (xn, xs), (yn, ys)):
            assert np.abs(got - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1.0)


def test_halpern_invariants(oracle_lib):
    """Eq. (hrpdhg): the anchor enters with weight 1/(k+2) and does not change
    the PDHG point; the reflection enters affinely with slope
    (k+1)/(k+2) (xhat - x); gamma = 0 is plain Halpern."""
    lp = gen.tiny_boxed_lp(5, 7, seed=9)
    o = _orc(lp)
    rng = np.random.default_rng(4)
    x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    x0, y0 = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    k = 6
    d = rng.standard_normal(lp.n)
    xh1, yh1, xn1, yn1 = o.lp_step(x, y, x0, y0, k, 0.2, 0.4, 1.0)
    xh2, yh2, xn2, yn2 = o.lp_step(x, y, x0 + d, y0, k, 0.2, 0.4, 1.0)
    np.testing.assert_array_equal(xh1, xh2)
    np.testing.assert_allclose(xn2 - xn1, d / (k + 2), atol=1e-13)
    _, _, xg0, yg0 = o.lp_step(x, y, x0, y0, k, 0.2, 0.4, 0.0)
    _, _, xg5, _ = o.lp_step(x, y, x0, y0, k, 0.2, 0.4, 0.5)
    np.testing.assert_allclose(xg0, (k + 1) / (k + 2) * xh1 + x0 / (k + 2), atol=1e-13)
    np.testing.assert_allclose(yg0, (k + 1) / (k + 2) * yh1 + y0 / (k + 2), atol=1e-13)
    np.testing.assert_allclose(xg5 - xg0, 0.5 * (k + 1) / (k + 2) * (xh1 - x), atol=1e-13)
    np.testing.assert_allclose(xn1 - xg0, 1.0 * (k + 1) / (k + 2) * (xh1 - x), atol=1e-13)


def test_fixed_point_residual_dense_m(oracle_lib):
    """r = ||z - zhat||_M with M = [[I/tau, A~'], [A~, I/sigma]] built
    explicitly; M is positive definite when tau sigma ||A~||^2 < 1."""
    lp = gen.planted_sparse_lp(20, 30, density=0.3, seed=7)
    o = _orc(lp)
    sc = o.scaling()
    at = _dense_scaled(lp, sc)
    tau, sigma = sc["eta"] / 2.0, sc["eta"] * 2.0
    mm = np.block([[np.eye(lp.n) / tau, at.T], [at, np.eye(lp.m) / sigma]])
    assert np.linalg.eigvalsh(mm).min() > 0
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    xh, yh = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    dz = np.concatenate([xh - x, yh - y])
    ref = np.sqrt(dz @ mm @ dz)
    assert abs(o.fixed_point_residual(x, y, xh, yh, tau, sigma) - ref) <= 1e-12 * ref


# ---------------------------------------------------------------------------
# scaling and step size


def test_pock_chambolle_norm_bound(oracle_lib):
    """Diagonal scaling with alpha = 1 (Pock & Chambolle) gives ||A~||_2 <= 1;
    the Lanczos estimate matches the dense 2-norm (from below: Ritz values
    never exceed the largest singular value)."""
    for seed in range(3):
        lp = gen.planted_sparse_lp(60, 90, density=0.1, seed=100 + seed)
        lp.val = lp.val * np.repeat(10.0 ** np.random.default_rng(seed).uniform(-2, 2, lp.m),
                                    np.diff(lp.rowptr))
        o = _orc(lp)
        sc = o.scaling()
        nrm = np.linalg.norm(_dense_scaled(lp, sc), 2)
        assert nrm <= 1.0 + 1e-12
        assert sc["norm_a"] <= nrm * (1 + 1e-12)
        assert sc["norm_a"] >= nrm * (1 - 1e-7)
        assert abs(sc["eta"] - 0.998 / sc["norm_a"]) <= 1e-15 * sc["eta"]


def test_lanczos_norm_on_structured_spectra(oracle_lib):
    """The grid incidence (two entries per column, a cluster of singular
    values at the top) and a dense Gaussian matrix: the estimate agrees with
    the dense 2-norm within 1e-7 after far fewer steps than the limit."""
    g = gen.grid_mincost_batch(batch=1, rows=10, cols=10, seed=3002).instance(0)
    d = gen.dense_planted_lp(80, 160, seed=7)
    for lp in (g, d):
        o = _orc(lp)
        sc = o.scaling()
        nrm = np.linalg.norm(_dense_scaled(lp, sc), 2)
        assert nrm * (1 - 1e-7) <= sc["norm_a"] <= nrm * (1 + 1e-12), (sc["norm_a"], nrm)
        assert 2 <= sc["power_iters"] < 300, sc["power_iters"]


def test_ruiz_equilibrates(oracle_lib):
    """Ruiz passes alone drive every row and column infinity-norm of
    D_r A D_c towards 1 (badly scaled input: rows spread over 1e-2..1e2)."""
    lp = gen.large_zipf_lp(m=2000, n=4000, seed=77)
    o = _orc(lp, ruiz_iters=20, pock_chambolle=0)
    sc = o.scaling()
    a = _dense_scaled(lp, sc)
    rmax = np.abs(a).max(axis=1)
    cmax = np.abs(a).max(axis=0)
    rmax, cmax = rmax[rmax > 0], cmax[cmax > 0]
    assert np.abs(rmax - 1).max() < 1e-3
    assert np.abs(cmax - 1).max() < 1e-3
    # the input spread is 4 orders of magnitude; D_r undoes it
    raw = np.abs(lp.to_dense()).max(axis=1)
    assert np.std(np.log10(raw[raw > 0])) > 1.0


def test_initial_weight(oracle_lib):
    """omega0 = ||c~|| / ||b~|| with b~_i the largest finite |bound| of row i."""
    lp = gen.planted_sparse_lp(seed=3)
    o = _orc(lp)
    sc, sv = o.scaling(), o.scaled_vectors()
    bt = np.maximum(np.where(np.isfinite(sv["lc"]), np.abs(sv["lc"]), 0),
                    np.where(np.isfinite(sv["uc"]), np.abs(sv["uc"]), 0))
    assert abs(sc["omega"] - np.linalg.norm(sv["c"]) / np.linalg.norm(bt)) <= 1e-13 * sc["omega"]
    np.testing.assert_allclose(sv["c"], sc["dc"] * lp.c, rtol=1e-15)
    np.testing.assert_allclose(sv["lv"], lp.lv / sc["dc"], rtol=1e-15)


# ---------------------------------------------------------------------------
# KKT


def test_kkt_planted_and_perturbed(oracle_lib):
    import oracle
    lp = gen.planted_sparse_lp(seed=1)
    r = oracle.kkt(lp, lp.x_star, lp.y_star)
    assert r["kkt"] < 1e-13
    assert abs(r["primal_obj"] - lp.v_star) < 1e-12 * (1 + abs(lp.v_star))
    # moving the primal off the equality rows shows up in the primal residual
    x = lp.x_star.copy()
    j = int(np.nonzero(lp.x_star)[0][0])
    x[j] += 0.01
    assert oracle.kkt(lp, x, lp.y_star)["rel_primal"] > 1e-6
    # moving the dual shows up in the dual residual or the gap
    y = lp.y_star.copy()
    y[np.isfinite(lp.lc) & np.isfinite(lp.uc)] *= 1.01
    r2 = oracle.kkt(lp, lp.x_star, y)
    assert max(r2["rel_dual"], r2["rel_gap"]) > 1e-6


def _highs(lp):
    from scipy.optimize import linprog
    a = lp.to_dense()
    eq = np.isfinite(lp.lc) & np.isfinite(lp.uc) & (lp.lc == lp.uc)
    up = np.isfinite(lp.uc) & ~eq
    lo = np.isfinite(lp.lc) & ~eq
    a_ub = np.vstack([a[up], -a[lo]])
    b_ub = np.concatenate([lp.uc[up], -lp.lc[lo]])
    bounds = [(None if not np.isfinite(l) else l, None if not np.isfinite(u) else u)
              for l, u in zip(lp.lv, lp.uv)]
    res = linprog(lp.c, A_ub=a_ub if len(b_ub) else None, b_ub=b_ub if len(b_ub) else None,
                  A_eq=a[eq] if eq.any() else None, b_eq=lp.lc[eq] if eq.any() else None,
                  bounds=bounds, method="highs",
                  options=dict(primal_feasibility_tolerance=1e-10, dual_feasibility_tolerance=1e-10))
    assert res.status == 0
    y = np.zeros(lp.m)
    if eq.any():
        y[eq] = res.eqlin.marginals
    nu = int(up.sum())
    mu = res.ineqlin.marginals if len(b_ub) else np.zeros(0)
    y[up] += mu[:nu]
    y[lo] -= mu[nu:]
    return res.x, y, res.fun


@pytest.mark.parametrize("seed", [0, 1])
def test_kkt_of_highs_solution(oracle_lib, seed):
    """The KKT error of HiGHS's primal-dual solution is ~0, and the oracle's
    sign conventions for y (R+ on >= rows, R- on <= rows) agree with it."""
    import oracle
    lp = gen.planted_sparse_lp(seed=seed)
    x, y, fun = _highs(lp)
    r = oracle.kkt(lp, x, y)
    assert r["kkt"] < 1e-8
    assert r["rel_gap"] < 1e-9
    assert oracle.kkt(lp, x, -y)["kkt"] > 1e-3


# ---------------------------------------------------------------------------
# full solves against independent optima


def _vertex_enumeration(lp):
    """min c'x over the polytope by enumerating basic solutions of G x <= h."""
    a = lp.to_dense()
    rows, rhs = [], []
    for i in range(lp.m):
        if np.isfinite(lp.uc[i]):
            rows.append(a[i]); rhs.append(lp.uc[i])
        if np.isfinite(lp.lc[i]):
            rows.append(-a[i]); rhs.append(-lp.lc[i])
    for j in range(lp.n):
        e = np.zeros(lp.n); e[j] = 1.0
        rows.append(e); rhs.append(lp.uv[j])
        rows.append(-e); rhs.append(-lp.lv[j])
    g, h = np.array(rows), np.array(rhs)
    best = np.inf
    for idx in itertools.combinations(range(len(h)), lp.n):
        gs = g[list(idx)]
        if abs(np.linalg.det(gs)) < 1e-10:
            continue
        x = np.linalg.solve(gs, h[list(idx)])
        if np.all(g @ x <= h + 1e-9):
            best = min(best, float(lp.c @ x))
    return best


@pytest.mark.parametrize("seed", range(6))
def test_solve_matches_vertex_enumeration(oracle_lib, seed):
    lp = gen.tiny_boxed_lp(3 + seed % 2, 4 + seed % 2, seed=200 + seed)
    ref = _vertex_enumeration(lp)
    x, y, r = _orc(lp, eps=1e-10).solve()
    assert r["status"] == 1
    assert abs(r["primal_obj"] - ref) <= 1e-7 * (1 + abs(ref))


def test_solve_small_lp_against_highs_and_planted(oracle_lib):
    """Small planted LP (m=200, n=400, 2% density): objective equals HiGHS's
    and the planted closed form V* = sum_eq y*_i b_i."""
    lp = gen.planted_sparse_lp(seed=0)
    _, _, fun = _highs(lp)
    assert abs(fun - lp.v_star) <= 1e-8 * (1 + abs(lp.v_star))
    x, y, r = _orc(lp, eps=1e-9).solve()
    assert r["status"] == 1
    assert abs(r["primal_obj"] - lp.v_star) <= 1e-7 * (1 + abs(lp.v_star))
    x, y, r = _orc(lp).solve()
    assert r["status"] == 1 and r["kkt"] <= 1e-4
    assert abs(r["primal_obj"] - lp.v_star) <= 1e-3 * (1 + abs(lp.v_star))


def test_solve_grid_flow_against_dijkstra(oracle_lib):
    """Capacities >= 5 >= k never bind, so the min-cost flow optimum is
    k * (shortest path length) on the arc costs (Dijkstra)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra
    g = gen.grid_mincost_batch(batch=3, rows=8, cols=8, seed=3001)
    tails, heads = g.meta["tails"], g.meta["heads"]
    for b in range(3):
        lp = g.instance(b)
        w = sp.csr_matrix((lp.c, (tails, heads)), shape=(g.m, g.m))
        dist = dijkstra(w, indices=int(g.meta["source"][b]))[int(g.meta["sink"][b])]
        ref = g.meta["supply"][b] * dist
        x, y, r = _orc(lp, eps=1e-9).solve()
        assert r["status"] == 1
        assert abs(r["primal_obj"] - ref) <= 1e-7 * (1 + ref)


def _water_filling(c, d, total=1.0, cap=0.1):
    lo, hi = -10.0, 10.0
    for _ in range(200):
        lam = 0.5 * (lo + hi)
        s = np.clip((lam - c) / d, 0.0, cap).sum()
        lo, hi = (lam, hi) if s < total else (lo, lam)
    return np.clip((0.5 * (lo + hi) - c) / d, 0.0, cap)


def test_qp_water_filling(oracle_lib):
    """Diagonal portfolio QP (F = 0): x_j = clip((lambda - c_j)/d_j, 0, 0.1)
    with lambda set so that sum x = 1 (Algorithm 2)."""
    p = gen.portfolio_qp_batch(batch=2, n=60, seed=9)
    for b in range(2):
        lp = gen.portfolio_instance(p, b)
        lp.q_factor = np.zeros((lp.n, 1))
        ref = _water_filling(lp.c, lp.q_diag)
        x, y, r = _orc(lp, eps=1e-10).solve()
        assert r["status"] == 1
        np.testing.assert_allclose(x, ref, atol=1e-6)
        vref = 0.5 * np.sum(lp.q_diag * ref ** 2) + lp.c @ ref
        assert abs(r["primal_obj"] - vref) <= 1e-8 * (1 + abs(vref))


def _qp_active_set(lp):
    """Strictly convex QP by enumerating which bound is active for every
    variable and row (lower, upper or none) and solving the KKT system."""
    q = gen.dense_from_csr(lp.n, lp.n, lp.q_rowptr, lp.q_colidx, lp.q_val)
    a = lp.to_dense()
    best = None
    choices = [(0, 1, 2)] * (lp.n + lp.m)
    for act in itertools.product(*choices):
        eqs_a, eqs_b = [], []
        ok = True
        for j in range(lp.n):
            if act[j] == 0 and np.isfinite(lp.lv[j]):
                e = np.zeros(lp.n); e[j] = 1; eqs_a.append(e); eqs_b.append(lp.lv[j])
            elif act[j] == 1 and np.isfinite(lp.uv[j]):
                e = np.zeros(lp.n); e[j] = 1; eqs_a.append(e); eqs_b.append(lp.uv[j])
            elif act[j] != 2:
                ok = False
        for i in range(lp.m):
            s = act[lp.n + i]
            if s == 0 and np.isfinite(lp.lc[i]):
                eqs_a.append(a[i]); eqs_b.append(lp.lc[i])
            elif s == 1 and np.isfinite(lp.uc[i]):
                eqs_a.append(a[i]); eqs_b.append(lp.uc[i])
            elif s != 2:
                ok = False
        if not ok:
            continue
        k = len(eqs_b)
        ea = np.array(eqs_a).reshape(k, lp.n)
        kkt = np.block([[q, ea.T], [ea, np.zeros((k, k))]])
        rhs = np.concatenate([-lp.c, np.array(eqs_b)])
        try:
            sol = np.linalg.solve(kkt, rhs)
        except np.linalg.LinAlgError:
            continue
        x = sol[: lp.n]
        if np.any(x < lp.lv - 1e-9) or np.any(x > lp.uv + 1e-9):
            continue
        ax = a @ x
        if np.any(ax < lp.lc - 1e-9) or np.any(ax > lp.uc + 1e-9):
            continue
        val = 0.5 * x @ q @ x + lp.c @ x
        if best is None or val < best[0] - 1e-12:
            best = (val, x)
    return best


@pytest.mark.parametrize("seed", range(3))
def test_qp_matches_active_set_enumeration(oracle_lib, seed):
    lp = gen.random_qp(2, 4, seed=300 + seed)
    val, xref = _qp_active_set(lp)
    x, y, r = _orc(lp, eps=1e-10).solve()
    assert r["status"] == 1
    assert abs(r["primal_obj"] - val) <= 1e-7 * (1 + abs(val))
    np.testing.assert_allclose(x, xref, atol=1e-5)


def test_qp_path_with_zero_q_reproduces_lp(oracle_lib):
    """rAPDHG with Q = 0 solves the LP: same optimum as r2HPDHG and V*."""
    lp = gen.planted_sparse_lp(seed=4)
    lpq = gen.planted_sparse_lp(seed=4)
    lpq.q_kind = "lowrank"
    lpq.q_factor = np.zeros((lp.n, 1))
    lpq.q_diag = np.zeros(lp.n)
    _, _, r_lp = _orc(lp, eps=1e-8).solve()
    _, _, r_qp = _orc(lpq, eps=1e-8).solve()
    assert r_qp["status"] == 1
    assert abs(r_qp["primal_obj"] - lp.v_star) <= 1e-6 * (1 + abs(lp.v_star))
    assert abs(r_lp["primal_obj"] - r_qp["primal_obj"]) <= 1e-6 * (1 + abs(lp.v_star))


# ---------------------------------------------------------------------------
# limits, warm start and validation


def test_iteration_limit_and_warm_start(oracle_lib):
    lp = gen.planted_sparse_lp(seed=2)
    x, y, r = _orc(lp, iteration_limit=10).solve()
    assert r["status"] == 4 and r["iterations"] == 10
    x1, y1, r1 = _orc(lp).solve()
    # warm start at the optimum: done at the first check
    x2, y2, r2 = _orc(lp).solve(lp.x_star, lp.y_star)
    assert r2["status"] == 1 and r2["iterations"] == 1
    assert r1["iterations"] > 64


def test_invalid_input_rejected(oracle_lib):
    import oracle
    lp = gen.planted_sparse_lp(seed=2)
    bad = gen.planted_sparse_lp(seed=2)
    bad.c = bad.c.copy(); bad.c[3] = np.nan
    with pytest.raises(ValueError):
        oracle.Oracle(bad)
    bad = gen.planted_sparse_lp(seed=2)
    bad.lv = bad.lv.copy(); bad.lv[0] = 5.0; bad.uv = bad.uv.copy(); bad.uv[0] = 1.0
    with pytest.raises(ValueError):
        oracle.Oracle(bad)
    bad = gen.planted_sparse_lp(seed=2)
    bad.colidx = bad.colidx.copy()
    r = int(np.argmax(np.diff(bad.rowptr) >= 2))
    s = bad.rowptr[r]
    bad.colidx[s], bad.colidx[s + 1] = bad.colidx[s + 1], bad.colidx[s]
    with pytest.raises(ValueError):
        oracle.Oracle(bad)
    oracle.Oracle(lp).close()


# ---------------------------------------------------------------------------
# unrolled iterations and their reverse pass


def test_unrolled_backward_matches_finite_differences(oracle_lib):
    """Reverse pass through T iterations with the frozen schedule against
    central differences (h = 1e-6) of the same frozen map."""
    lp = gen.tiny_boxed_lp(4, 6, seed=31)
    lp.uv[:2] = INF
    T = 150
    o = _orc(lp)
    x, y, sr, sw = o.unrolled(T)
    rng = np.random.default_rng(0)
    wx, wy = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    gc, glc, guc = o.backward(T, sr, sw, wx, wy)
    h = 1e-6

    def loss(c=None, lc=None, uc=None):
        q = gen.tiny_boxed_lp(4, 6, seed=31)
        q.uv[:2] = INF
        if c is not None: q.c = c
        if lc is not None: q.lc = lc
        if uc is not None: q.uc = uc
        xx, yy, _, _ = _orc(q).unrolled(T, sr, sw)
        return wx @ xx + wy @ yy

    for j in range(lp.n):
        e = np.zeros(lp.n); e[j] = h
        fd = (loss(c=lp.c + e) - loss(c=lp.c - e)) / (2 * h)
        assert abs(fd - gc[j]) <= 1e-6 * (1 + abs(fd))
    for i in range(lp.m):
        e = np.zeros(lp.m); e[i] = h
        if np.isfinite(lp.lc[i]) and lp.lc[i] != lp.uc[i]:
            fd = (loss(lc=lp.lc + e) - loss(lc=lp.lc - e)) / (2 * h)
            assert abs(fd - glc[i]) <= 1e-6 * (1 + abs(fd))
        if np.isfinite(lp.uc[i]) and lp.lc[i] != lp.uc[i]:
            fd = (loss(uc=lp.uc + e) - loss(uc=lp.uc - e)) / (2 * h)
            assert abs(fd - guc[i]) <= 1e-6 * (1 + abs(fd))


def test_unrolled_envelope_gradient(oracle_lib):
    """At convergence d(c'x*)/dc = x* (envelope theorem): the reverse pass of
    the value c'x_T plus its explicit term gives the solution itself."""
    lp = gen.planted_sparse_lp(40, 80, density=0.1, seed=8)
    o = _orc(lp)
    xs, ys, r = _orc(lp, eps=1e-9).solve()
    T = int(r["iterations"]) + 200
    x, y, sr, sw = o.unrolled(T)
    gc, _, _ = o.backward(T, sr, sw, lp.c, np.zeros(lp.m))
    grad = x + gc
    assert np.abs(grad - xs).max() <= 1e-4 * (1 + np.abs(xs).max())


def test_unrolled_qp_backward_matches_finite_differences(oracle_lib):
    """Reverse pass of unrolled rAPDHG (frozen schedule) against central
    differences in c and in the diagonal d of Q = F F' + diag(d)."""
    p = gen.portfolio_qp_batch(batch=1, n=12, rank=3, seed=4800)
    base = gen.portfolio_instance(p, 0)
    T = 120
    o = _orc(base)
    x, y, sr, sw = o.unrolled_qp(T)
    assert sr.sum() >= 1          # the schedule contains restarts
    rng = np.random.default_rng(2)
    wx, wy = rng.standard_normal(base.n), rng.standard_normal(base.m)
    gc, glc, guc, gd = o.backward_qp(T, sr, sw, wx, wy)
    h = 1e-6

    sc = o.scaling()

    def loss(c=None, d=None):
        q = gen.portfolio_instance(p, 0)
        if c is not None: q.c = c
        if d is not None: q.q_diag = d
        oq = _orc(q)
        oq.pin_steps(sc["eta"], sc["norm_q"])   # frozen step sizes
        xx, yy, _, _ = oq.unrolled_qp(T, sr, sw)
        return wx @ xx + wy @ yy

    for j in range(base.n):
        e = np.zeros(base.n); e[j] = h
        fd = (loss(c=base.c + e) - loss(c=base.c - e)) / (2 * h)
        assert abs(fd - gc[j]) <= 1e-6 * (1 + abs(fd)), ("c", j, fd, gc[j])
        fd = (loss(d=base.q_diag + e) - loss(d=base.q_diag - e)) / (2 * h)
        assert abs(fd - gd[j]) <= 1e-6 * (1 + abs(fd)), ("d", j, fd, gd[j])


def test_unrolled_qp_envelope(oracle_lib):
    """At convergence d(V)/dc = x* and d(V)/dd = x*^2 / 2 for
    V = 1/2 x'Qx + c'x (envelope theorem)."""
    p = gen.portfolio_qp_batch(batch=1, n=30, rank=4, seed=4900)
    lp = gen.portfolio_instance(p, 0)
    xs, ys, r = _orc(lp, eps=1e-10).solve()
    T = int(r["iterations"]) + 300
    o = _orc(lp)
    x, y, sr, sw = o.unrolled_qp(T)
    qx = lp.q_factor @ (lp.q_factor.T @ x) + lp.q_diag * x
    # dV/dx_T = Q x_T + c; chain through the reverse pass, plus the explicit terms
    gc, _, _, gd = o.backward_qp(T, sr, sw, qx + lp.c, np.zeros(lp.m))
    np.testing.assert_allclose(gc + x, xs, atol=2e-4)
    np.testing.assert_allclose(gd + 0.5 * x * x, 0.5 * xs * xs, atol=2e-4)


# ---------------------------------------------------------------------------
# ||Q~||_2 (Algorithm 2's step sizes use it; the power iteration of reading R11)


def _splitmix64(x: int) -> int:
    """SplitMix64 (Steele, Lea and Flood, 2014): first output of the generator
    seeded with x."""
    mask = (1 << 64) - 1
    z = (x + 0x9E3779B97F4A7C15) & mask
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
    return z ^ (z >> 31)


def _dense_q(lp):
    if lp.q_kind == "lowrank":
        return lp.q_factor @ lp.q_factor.T + np.diag(lp.q_diag)
    return gen.dense_from_csr(lp.n, lp.n, lp.q_rowptr, lp.q_colidx, lp.q_val)


def _norm_q_cases():
    p = gen.portfolio_qp_batch(batch=1, n=80, rank=6, seed=41)
    dense_q = gen.random_qp(6, 12, seed=5)   # G G' + 0.1 I stored with every entry
    return [gen.portfolio_instance(p, 0), gen.random_qp(5, 9, seed=3),
            gen.infeasible_qp("duplicate_row", seed=2), dense_q]


def test_splitmix64_published_outputs():
    """The generator's first outputs for seed 0 as published with it."""
    assert _splitmix64(0) == 0xE220A8397B1DCDAF
    assert _splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


def test_norm_q_matches_dense_eigenvalue(oracle_lib):
    """The converged estimate is the largest eigenvalue of Q~ = D_c Q D_c (its
    2-norm, Q~ being PSD), approached from below. With Rayleigh quotients
    converging like rho^(2k), rho = lambda_2 / lambda_1, the stopping test
    (relative change <= 1e-7) leaves a relative error of at most about
    1e-7 rho^2 / (1 - rho^2); the bar adds a factor 2. A square root of the
    eigenvalue, or a Q~ scaled by D_c once instead of on both sides, fails it."""
    for lp in _norm_q_cases():
        sc = _orc(lp).scaling()
        qs = sc["dc"][:, None] * _dense_q(lp) * sc["dc"][None, :]
        ev = np.linalg.eigvalsh(qs)
        lam, lam2 = ev[-1], ev[-2]
        assert abs(np.linalg.norm(qs, 2) - lam) <= 1e-12 * lam
        rho2 = (lam2 / lam) ** 2
        bar = 2e-7 * rho2 / (1 - rho2) + 1e-13
        assert lam * (1 - bar) <= sc["norm_q"] <= lam * (1 + 1e-12), (sc["norm_q"], lam, bar)
        assert abs(sc["norm_q"] - lam) > 1e-3 * lam or abs(np.sqrt(lam) - lam) > 1e-3 * lam


def test_norm_q_rayleigh_quotients_of_the_start_vector(oracle_lib):
    """Stopped after k power steps, the estimate is the Rayleigh quotient of
    Q~^(k-1) v0: m_(2k-1) / m_(2k-2) with moments m_j = v0' Q~^j v0, v0 the
    normalised start vector v0_j = 0.5 + u_j (u_j from SplitMix64 at counter
    j, the top 53 bits). It rises monotonically towards lambda_max. Returning
    |Q~ v| (= sqrt(m_2k / m_(2k-2))) or its square root fails it."""
    for lp in _norm_q_cases():
        v0 = np.array([0.5 + (_splitmix64(j) >> 11) * 2.0 ** -53 for j in range(lp.n)])
        v0 /= np.linalg.norm(v0)
        sc = _orc(lp).scaling()
        qs = sc["dc"][:, None] * _dense_q(lp) * sc["dc"][None, :]
        mom = [v0 @ v0]
        w = v0.copy()
        for _ in range(8):
            w = qs @ w
            mom.append(v0 @ w)
        prev = -np.inf
        for k in range(1, 5):
            est = _orc(lp, power_max_iters=k).scaling()["norm_q"]
            ref = mom[2 * k - 1] / mom[2 * k - 2]
            assert abs(est - ref) <= 1e-12 * ref, (k, est, ref)
            assert abs(np.sqrt(mom[2 * k] / mom[2 * k - 2]) - ref) > 1e-9 * ref
            assert est >= prev * (1 - 1e-14)
            prev = est
        assert prev <= np.linalg.eigvalsh(qs)[-1] * (1 + 1e-12)


def test_results_do_not_depend_on_thread_count(oracle_lib):
    """The products may run on several threads (rows of A~, columns of A~'
    through a column-major copy); every entry is summed in the same order, so
    a solve and the scaling are bitwise equal on 1 and 4 threads."""
    lp = gen.large_zipf_lp(m=3000, n=6000, kmax=300, seed=91)
    out = []
    for t in (1, 4):
        oracle_lib.set_threads(t)
        o = _orc(lp, iteration_limit=700)
        sc = o.scaling()
        x, y, r = o.solve()
        out.append((sc["eta"], sc["power_iters"], x, y, r["iterations"], r["primal_obj"]))
    oracle_lib.set_threads(1)
    a, b = out
    assert a[0] == b[0] and a[1] == b[1] and a[4] == b[4] and a[5] == b[5]
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_array_equal(a[3], b[3])
