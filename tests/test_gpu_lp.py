"""GPU parity of the r2HPDHG path against the CPU oracle (through the C ABI).

Bars: one iteration within 1e-12 relative (max-norm per output vector); the
scaling vectors within 1e-12; a full solve reaches relative KKT <= 1e-4 with
the objective within 1e-6 relative of the oracle's."""

import sys

import numpy as np
import pytest

import gen
from gpu_util import rel_inf, to_np

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-12


@pytest.fixture(scope="module")
def pdhg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_09734_amd.solver as s
    return s


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _step_case(pdhg, oracle_lib, lp, seeds=(0, 1), ks=(0, 5, 1000), compare_eta=True):
    orc = oracle_lib.Oracle(lp) if compare_eta else oracle_lib.Oracle(lp, power_max_iters=1)
    sc = orc.scaling()
    with pdhg.Solver.from_lp(lp) as s:
        gs = s.scaling()
        assert rel_inf(to_np(gs["dc"]), sc["dc"]) <= STEP_TOL
        if lp.m:
            assert rel_inf(to_np(gs["dr"]), sc["dr"]) <= STEP_TOL
        if compare_eta:
            assert abs(gs["eta"] - sc["eta"]) <= 1e-10 * sc["eta"]
            assert gs["power_iters"] == sc["power_iters"]
        assert abs(gs["omega"] - sc["omega"]) <= 1e-10 * sc["omega"]
        for seed in seeds:
            rng = np.random.default_rng(seed)
            x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
            x0, y0 = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
            for k in ks:
                tau, sigma = sc["eta"] / sc["omega"] * (1 + seed), sc["eta"] * sc["omega"]
                got = s.debug_step(x, y, x0, y0, k, tau, sigma)
                ref = orc.lp_step(x, y, x0, y0, k, tau, sigma)
                for name, g, r in zip(("xhat", "yhat", "xnew", "ynew"), got, ref):
                    err = rel_inf(to_np(g), r)
                    assert err <= STEP_TOL, (name, seed, k, err)
                # the plain iteration between checks (its own product layouts)
                got = s.debug_plain_step(x, y, x0, y0, k, tau, sigma)
                for name, g, r in zip(("xnew", "ynew"), got, ref[2:]):
                    err = rel_inf(to_np(g), r)
                    assert err <= STEP_TOL, ("plain " + name, seed, k, err)


def test_step_parity_small_lp(pdhg, oracle_lib):
    _say("case: step parity, planted m=200 n=400")
    _step_case(pdhg, oracle_lib, gen.planted_sparse_lp(seed=0))


def test_step_parity_mixed_bounds(pdhg, oracle_lib):
    _say("case: step parity, boxed LP with every bound kind")
    lp = gen.tiny_boxed_lp(37, 61, seed=3)
    lp.lv[::5] = -np.inf
    lp.uv[2::7] = np.inf
    _step_case(pdhg, oracle_lib, lp)


def _skewed_lp(seed=5):
    """Rows and columns of very different lengths (every lane class, ragged
    tails): a few dense rows/columns plus many 1-2 entry ones, empty rows and
    columns, free rows."""
    rng = np.random.default_rng(seed)
    m, n = 1500, 3100
    rows, cols = [], []
    for i in range(m):
        k = int(min(n, rng.zipf(1.6)))
        if i % 97 == 0:
            k = 0
        rows += [i] * k
        cols += list(rng.choice(n, size=k, replace=False))
    dense_col = 7
    rows += list(range(0, m, 2))
    cols += [dense_col] * len(range(0, m, 2))
    rows += [3] * 2500
    cols += list(rng.choice(n, size=2500, replace=False))
    key = np.unique(np.asarray(rows, np.int64) * n + np.asarray(cols, np.int64))
    r, c = key // n, (key % n).astype(np.int32)
    rowptr = np.zeros(m + 1, np.int32)
    np.cumsum(np.bincount(r, minlength=m), out=rowptr[1:])
    val = rng.standard_normal(len(c)) * 10.0 ** rng.uniform(-2, 2, len(c))
    lc = np.where(rng.random(m) < 0.5, -rng.random(m), -np.inf)
    uc = np.where(rng.random(m) < 0.5, rng.random(m), np.inf)
    lc[::11] = -np.inf
    uc[::11] = np.inf
    lv = np.where(rng.random(n) < 0.7, 0.0, -np.inf)
    uv = np.where(rng.random(n) < 0.3, 3.0, np.inf)
    return gen.LP(m, n, rowptr, c, val, rng.standard_normal(n), lc, uc, lv, uv)


def test_step_parity_skewed_lengths(pdhg, oracle_lib):
    _say("case: step parity, skewed row/column lengths")
    _step_case(pdhg, oracle_lib, _skewed_lp())


def test_step_parity_grid_flow(pdhg, oracle_lib):
    _say("case: step parity, grid min-cost flow")
    _step_case(pdhg, oracle_lib, gen.grid_mincost_batch(batch=1, seed=3000).instance(0))


def test_step_parity_no_rows(pdhg, oracle_lib):
    _say("case: step parity, m=0")
    n = 300
    lp = gen.LP(0, n, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0),
                np.linspace(-1, 1, n), np.zeros(0), np.zeros(0), np.full(n, -2.0), np.full(n, 5.0))
    _step_case(pdhg, oracle_lib, lp, ks=(0, 3))


# Product layouts of the plain iterations, forced on small LPs: LDS panels of
# y for the long rows of A~' (many panels, sub-rows longer than a 64-entry
# chunk, every row in the panels) and x_ext entries staged in LDS by the dual
# product.
PANEL_LAYOUTS = {
    "many_panels": dict(panel_rows=64, panel_min_len=4, panel_wgs=2, hot_cols=100),
    "all_rows_in_panels": dict(panel_rows=1000, panel_min_len=0, panel_wgs=1, hot_cols=16384),
    "wide_panels": dict(panel_rows=16384, panel_min_len=16, panel_wgs=4, hot_cols=0),
    "widest_panels": dict(panel_rows=20480, panel_min_len=8, panel_wgs=3, hot_cols=20480),
    "hot_columns_only": dict(panel_rows=0, hot_cols=37),
}


def _layout_lp(name):
    if name == "skewed":
        return _skewed_lp()
    if name == "zipf":
        return gen.large_zipf_lp(m=3000, n=6000, kmax=400, seed=83)
    return gen.grid_mincost_batch(batch=1, seed=3001).instance(0)


@pytest.mark.parametrize("layout", sorted(PANEL_LAYOUTS))
@pytest.mark.parametrize("name", ["skewed", "zipf", "grid"])
def test_plain_step_parity_panel_layouts(pdhg, oracle_lib, name, layout):
    """One plain iteration through each product layout against the oracle;
    with the panels off, the hot-column dual product equals the standard one
    bit for bit (same summation order)."""
    _say(f"case: plain step parity, {name} LP, layout {layout}")
    lp = _layout_lp(name)
    orc = oracle_lib.Oracle(lp)
    sc = orc.scaling()
    rng = np.random.default_rng(11)
    x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    x0, y0 = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    with pdhg.Solver.from_lp(lp, **PANEL_LAYOUTS[layout]) as s, \
            pdhg.Solver.from_lp(lp, panel_rows=0, hot_cols=0) as plain:
        for k in (0, 9):
            tau, sigma = sc["eta"] / sc["omega"], sc["eta"] * sc["omega"]
            ref = orc.lp_step(x, y, x0, y0, k, tau, sigma)
            got = s.debug_plain_step(x, y, x0, y0, k, tau, sigma)
            for nm, g, r in zip(("xnew", "ynew"), got, ref[2:]):
                err = rel_inf(to_np(g), r)
                assert err <= STEP_TOL, (nm, k, err)
            if PANEL_LAYOUTS[layout]["panel_rows"] == 0:
                base = plain.debug_plain_step(x, y, x0, y0, k, tau, sigma)
                for g, b in zip(got, base):
                    np.testing.assert_array_equal(to_np(g), to_np(b))


@pytest.mark.parametrize("layout", ["many_panels", "all_rows_in_panels"])
def test_solve_parity_panel_layouts(pdhg, oracle_lib, layout):
    """Full solves whose plain iterations run through the panels and hot
    columns: optimal at KKT <= 1e-4, objective within 1e-6 of the oracle's,
    the reported KKT error that of the returned point, and bitwise repeatable."""
    lp = gen.planted_sparse_lp(m=300, n=600, density=0.05, seed=7)
    _say(f"case: full solve parity, planted m=300 n=600, layout {layout}")
    xo, yo, ro = oracle_lib.Oracle(lp).solve()
    with pdhg.Solver.from_lp(lp, **PANEL_LAYOUTS[layout]) as s:
        xg, yg, rg = s.solve()
        x2, y2, r2 = s.solve()
    _say(f"  iterations gpu={rg['iterations']} oracle={ro['iterations']}")
    assert rg["status_name"] == "optimal" and rg["kkt_rel"] <= 1e-4
    assert rg["iterations"] == ro["iterations"]
    assert abs(rg["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))
    kg = oracle_lib.kkt(lp, to_np(xg), to_np(yg))
    assert abs(kg["kkt"] - rg["kkt_rel"]) <= 1e-9 + 1e-6 * kg["kkt"]
    np.testing.assert_array_equal(to_np(xg), to_np(x2))
    np.testing.assert_array_equal(to_np(yg), to_np(y2))
    assert rg["iterations"] == r2["iterations"]


def test_solve_parity_small_lp(pdhg, oracle_lib):
    for seed in (0, 1, 2):
        _say(f"case: full solve parity, planted m=200 n=400 seed={seed}")
        lp = gen.planted_sparse_lp(seed=seed)
        xo, yo, ro = oracle_lib.Oracle(lp).solve()
        with pdhg.Solver.from_lp(lp) as s:
            xg, yg, rg = s.solve()
        _say(f"  iterations gpu={rg['iterations']} oracle={ro['iterations']} "
             f"restarts gpu={rg['restarts']} oracle={ro['restarts']}")
        assert rg["status_name"] == "optimal" and rg["kkt_rel"] <= 1e-4
        assert ro["status"] == 1 and ro["kkt"] <= 1e-4
        assert rg["iterations"] == ro["iterations"] and rg["restarts"] == ro["restarts"]
        assert abs(rg["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))
        # the reported KKT error is that of the returned point
        kg = oracle_lib.kkt(lp, to_np(xg), to_np(yg))
        assert abs(kg["kkt"] - rg["kkt_rel"]) <= 1e-9 + 1e-6 * kg["kkt"]


def test_solve_parity_zipf_long_columns(pdhg, oracle_lib):
    """Zipf column degrees with columns longer than the SELL limit, so A~'
    has long rows (lane groups with a butterfly sum)."""
    for (m, n, seed) in ((1000, 2000, 79), (800, 1600, 81)):
        _say(f"case: full solve parity, Zipf planted m={m} n={n} seed={seed}")
        lp = gen.large_zipf_lp(m=m, n=n, kmax=300, seed=seed)
        assert (np.bincount(lp.colidx, minlength=n) > 64).sum() > 10
        xo, yo, ro = oracle_lib.Oracle(lp).solve()
        with pdhg.Solver.from_lp(lp) as s:
            xg, yg, rg = s.solve()
        _say(f"  iterations gpu={rg['iterations']} oracle={ro['iterations']}")
        assert rg["status_name"] == "optimal" and rg["kkt_rel"] <= 1e-4
        assert rg["iterations"] == ro["iterations"]
        assert abs(rg["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))
        kg = oracle_lib.kkt(lp, to_np(xg), to_np(yg))
        assert kg["kkt"] <= 1e-4
        assert abs(kg["kkt"] - rg["kkt_rel"]) <= 1e-9 + 1e-6 * kg["kkt"]


def test_solve_parity_grid_flow(pdhg, oracle_lib):
    g = gen.grid_mincost_batch(batch=2, seed=3000)
    for b in range(2):
        _say(f"case: full solve parity, grid min-cost flow instance {b}")
        lp = g.instance(b)
        xo, yo, ro = oracle_lib.Oracle(lp).solve()
        with pdhg.Solver.from_lp(lp) as s:
            xg, yg, rg = s.solve()
        assert rg["status_name"] == "optimal"
        assert rg["iterations"] == ro["iterations"]
        assert abs(rg["primal_obj"] - ro["primal_obj"]) <= 1e-6 * (1 + abs(ro["primal_obj"]))


def test_solve_is_deterministic(pdhg):
    _say("case: bitwise determinism")
    lp = gen.planted_sparse_lp(seed=1)
    with pdhg.Solver.from_lp(lp) as s:
        x1, y1, r1 = s.solve()
        x1, y1 = to_np(x1), to_np(y1)
        x2, y2, r2 = s.solve()
    np.testing.assert_array_equal(x1, to_np(x2))
    np.testing.assert_array_equal(y1, to_np(y2))
    assert r1["iterations"] == r2["iterations"]


def test_limits_and_warm_start(pdhg, oracle_lib):
    _say("case: iteration limits and warm start")
    lp = gen.planted_sparse_lp(seed=2)
    for limit in (1, 10, 64, 65, 130):
        xo, yo, ro = oracle_lib.Oracle(lp, iteration_limit=limit).solve()
        with pdhg.Solver.from_lp(lp, iteration_limit=limit) as s:
            xg, yg, rg = s.solve()
        assert rg["status"] == ro["status"] == 4
        assert rg["iterations"] == ro["iterations"] == limit
        assert rel_inf(to_np(xg), xo) <= 1e-10 and rel_inf(to_np(yg), yo) <= 1e-10
    with pdhg.Solver.from_lp(lp) as s:
        xg, yg, rg = s.solve(lp.x_star, lp.y_star)
    assert rg["status_name"] == "optimal" and rg["iterations"] == 1
    # no graph replay: same iterates
    with pdhg.Solver.from_lp(lp, use_graph=0) as s:
        xa, ya, ra = s.solve()
    with pdhg.Solver.from_lp(lp) as s:
        xb, yb, rb = s.solve()
    np.testing.assert_array_equal(to_np(xa), to_np(xb))


def test_update_data_matches_fresh_handle(pdhg):
    _say("case: update_data")
    lp = gen.planted_sparse_lp(seed=3)
    lp2 = gen.planted_sparse_lp(seed=3)
    lp2.c = lp.c * 1.5 + 0.1
    with pdhg.Solver.from_lp(lp) as s:
        s.update_data(c=lp2.c)
        xa, ya, ra = s.solve()
    with pdhg.Solver.from_lp(lp2) as s:
        xb, yb, rb = s.solve()
    np.testing.assert_array_equal(to_np(xa), to_np(xb))
    assert ra["iterations"] == rb["iterations"]


def test_invalid_inputs_rejected(pdhg):
    _say("case: invalid inputs")
    from paper_2412_09734_amd._capi import PdhgError
    lp = gen.planted_sparse_lp(seed=4)
    bad = dict(m=lp.m, n=lp.n, rowptr=lp.rowptr, colidx=lp.colidx, val=lp.val, c=lp.c,
               lc=lp.lc, uc=lp.uc, lv=lp.lv, uv=lp.uv)
    c = lp.c.copy(); c[5] = np.nan
    with pytest.raises(PdhgError) as e:
        pdhg.Solver(**{**bad, "c": c})
    assert e.value.code == -2
    ci = lp.colidx.copy()
    r = int(np.argmax(np.diff(lp.rowptr) >= 2))
    ci[lp.rowptr[r]], ci[lp.rowptr[r] + 1] = ci[lp.rowptr[r] + 1], ci[lp.rowptr[r]]
    with pytest.raises(PdhgError) as e:
        pdhg.Solver(**{**bad, "colidx": ci})
    assert e.value.code == -2
    lv = lp.lv.copy(); lv[0] = 1.0
    uv = lp.uv.copy(); uv[0] = 0.5
    with pytest.raises(PdhgError) as e:
        pdhg.Solver(**{**bad, "lv": lv, "uv": uv})
    assert e.value.code == -2
    v = lp.val.copy(); v[0] = np.inf
    with pytest.raises(PdhgError) as e:
        pdhg.Solver(**{**bad, "val": v})
    assert e.value.code == -2


@pytest.mark.timeout(600)
def test_step_parity_large_zipf_lp(pdhg, oracle_lib):
    """Full-size sparse LP (m=1e6, n=2e6, Zipf columns): one iteration and the
    scaling, in the layout and launch configuration the benchmark times."""
    _say("case: step parity at full size m=1e6 n=2e6 (generation + oracle take ~1 min)")
    lp = gen.large_zipf_lp(seed=1000)
    _say(f"  generated nnz={lp.nnz}")
    _step_case(pdhg, oracle_lib, lp, seeds=(0,), ks=(7,), compare_eta=False)


@pytest.mark.parametrize("kind,m,n,seed", [("duplicate_row", 60, 120, 0), ("boxed_sum", 30, 50, 3),
                                           ("unbounded", 400, 800, 1), ("duplicate_row", 2000, 4000, 5),
                                           ("unbounded", 2000, 4000, 6)])
def test_infeasibility_certificates_match_oracle(pdhg, oracle_lib, kind, m, n, seed):
    """Status, iteration of the certifying check and the returned ray (dual
    ray in y for an infeasible LP, primal ray in x for an unbounded one)."""
    _say(f"case: infeasibility detection, {kind} m={m} n={n} seed={seed}")
    lp = gen.infeasible_lp(kind, m, n, seed=seed)
    xo, yo, ro = oracle_lib.Oracle(lp, iteration_limit=100000).solve()
    with pdhg.Solver.from_lp(lp, iteration_limit=100000) as s:
        xg, yg, rg = s.solve()
    _say(f"  status gpu={rg['status_name']} oracle={ro['status_name']} "
         f"iterations gpu={rg['iterations']} oracle={ro['iterations']}")
    want = "dual_infeasible" if kind == "unbounded" else "primal_infeasible"
    assert ro["status_name"] == want and rg["status_name"] == want
    # the same iterates cross the 1e-8 threshold at the same check
    assert rg["iterations"] == ro["iterations"]
    if want == "primal_infeasible":
        assert rel_inf(to_np(yg), yo) <= 1e-8
    else:
        assert rel_inf(to_np(xg), xo) <= 1e-8


def test_infeasibility_switches(pdhg):
    _say("case: infeasibility tests switched off run to the iteration limit")
    lp = gen.infeasible_lp("duplicate_row", 60, 120, seed=0)
    with pdhg.Solver.from_lp(lp, iteration_limit=3000, eps_primal_infeasible=0.0) as s:
        assert s.solve()[2]["status_name"] == "iteration_limit"
    lp = gen.infeasible_lp("unbounded", 60, 120, seed=0)
    with pdhg.Solver.from_lp(lp, iteration_limit=3000, eps_dual_infeasible=0.0) as s:
        assert s.solve()[2]["status_name"] == "iteration_limit"


@pytest.mark.timeout(900)
def test_infeasibility_certificate_full_size(pdhg):
    """The 1M x 2M Zipf LP with one equality row duplicated at a moved
    right-hand side: the solve stops with a dual ray, checked here as a
    Farkas certificate with scipy's sparse products (the oracle cannot
    finish a solve of this size)."""
    import scipy.sparse as sp
    _say("case: infeasibility certificate at full size m=1e6+1 n=2e6 (generation ~30 s)")
    lp = gen.contradict_row(gen.large_zipf_lp(seed=1000), seed=1)
    with pdhg.Solver.from_lp(lp, iteration_limit=200000) as s:
        _, yg, rg = s.solve()
    _say(f"  status={rg['status_name']} iterations={rg['iterations']}")
    assert rg["status_name"] == "primal_infeasible"
    y = to_np(yg)
    ge = np.isfinite(lp.lc) & ~np.isfinite(lp.uc)
    le = ~np.isfinite(lp.lc) & np.isfinite(lp.uc)
    assert np.min(y[ge], initial=0.0) >= -1e-8 and np.max(y[le], initial=0.0) <= 1e-8
    pos, neg = (y > 0) & np.isfinite(lp.lc), (y < 0) & np.isfinite(lp.uc)
    b_y = np.dot(lp.lc[pos], y[pos]) + np.dot(lp.uc[neg], y[neg])
    A = sp.csr_matrix((lp.val, lp.colidx, lp.rowptr), shape=(lp.m, lp.n))
    g = A.T @ y
    # Farkas: feasible x have y'Ax >= b(y); over x >= 0 with u_v = 10 on half
    # the columns, y'Ax = g'x is at most sum of u_v max(g, 0) over the boxed
    # columns when g <= 0 (up to 1e-8) on the others. The ray is scaled so
    # that the margin b(y) - that sum is 1.
    boxed = np.isfinite(lp.uv)
    assert np.max(g[~boxed], initial=0.0) <= 1e-8
    margin = b_y - np.sum(lp.uv[boxed] * np.maximum(g[boxed], 0.0))
    assert abs(margin - 1.0) <= 1e-6, margin


@pytest.mark.parametrize("name", ["planted", "boxed", "grid", "dense"])
def test_feasibility_polishing_matches_oracle(pdhg, oracle_lib, name):
    """Polishing after an optimal solve: the same phase lengths as the oracle,
    the same polished point, and its reported KKT terms are those of the
    returned point."""
    _say(f"case: feasibility polishing parity, {name}")
    if name == "planted":
        lp = gen.planted_sparse_lp(200, 400, seed=11)
    elif name == "boxed":
        lp = gen.tiny_boxed_lp(12, 20, seed=13)
    elif name == "grid":
        lp = gen.grid_mincost_batch(batch=1, rows=6, cols=6, seed=14).instance(0)
    else:
        lp = gen.dense_planted_lp(150, 300, seed=2001)
    xo, yo, ro = oracle_lib.Oracle(lp, feasibility_polishing=1).solve()
    with pdhg.Solver.from_lp(lp, feasibility_polishing=1) as s:
        xg, yg, rg = s.solve()
    _say(f"  polish iterations gpu={rg['polish_iterations']} oracle={ro['polish_iterations']} "
         f"rel_p={rg['rel_primal_res']:.2e} rel_d={rg['rel_dual_res']:.2e} gap={rg['rel_gap']:.2e}")
    assert rg["status_name"] == "optimal" and ro["status_name"] == "optimal"
    assert rg["polish_iterations"] == ro["polish_iterations"] > 0
    assert rg["iterations"] == ro["iterations"]
    assert rg["rel_primal_res"] <= 1e-6 and rg["rel_dual_res"] <= 1e-6
    assert rel_inf(to_np(xg), xo) <= 1e-8
    assert rel_inf(to_np(yg), yo) <= 1e-8
    kg = oracle_lib.kkt(lp, to_np(xg), to_np(yg))
    for a, b in (("rel_primal_res", "rel_primal"), ("rel_dual_res", "rel_dual"), ("rel_gap", "rel_gap")):
        assert abs(rg[a] - kg[b]) <= 1e-12 + 1e-6 * kg[b], (a, rg[a], kg[b])
    # the handle's data is restored: a second solve without polishing is the plain one
    with pdhg.Solver.from_lp(lp) as s:
        _, _, r_plain = s.solve()
    assert r_plain["iterations"] == rg["iterations"] - rg["polish_iterations"]


@pytest.mark.timeout(900)
def test_feasibility_polishing_full_size(pdhg):
    """The 1M x 2M Zipf LP solved to 1e-3 and polished: the returned point's
    relative primal and dual residuals, computed here with scipy from the LP's
    data, are <= 1e-6 and equal the reported ones."""
    import scipy.sparse as sp
    _say("case: feasibility polishing at full size m=1e6 n=2e6, eps 1e-3")
    lp = gen.large_zipf_lp(seed=1000)
    with pdhg.Solver.from_lp(lp, eps=1e-3, feasibility_polishing=1) as s:
        xg, yg, rg = s.solve()
    _say(f"  iterations={rg['iterations']} polish={rg['polish_iterations']} rel_p={rg['rel_primal_res']:.2e} "
         f"rel_d={rg['rel_dual_res']:.2e} gap={rg['rel_gap']:.2e}")
    assert rg["status_name"] == "optimal"
    x, y = to_np(xg), to_np(yg)
    A = sp.csr_matrix((lp.val, lp.colidx, lp.rowptr), shape=(lp.m, lp.n))
    ax = A @ x
    rp = ax - np.clip(ax, lp.lc, lp.uc)
    b = np.maximum(np.where(np.isfinite(lp.lc), np.abs(lp.lc), 0.0), np.where(np.isfinite(lp.uc), np.abs(lp.uc), 0.0))
    rel_p = np.linalg.norm(rp) / (1 + np.linalg.norm(b))
    # x = D_c xhat with xhat in [l_v, u_v] / D_c: within an ulp of the box
    assert np.all(x >= lp.lv - 1e-12 * (1 + np.abs(lp.lv))) and np.all(x <= lp.uv + 1e-12 * (1 + np.abs(lp.uv)))
    g = lp.c - A.T @ y
    lo_f, up_f = np.isfinite(lp.lv), np.isfinite(lp.uv)
    allowed = np.where(lo_f & up_f, g, np.where(lo_f, np.maximum(g, 0), np.where(up_f, np.minimum(g, 0), 0)))
    rel_d = np.linalg.norm(g - allowed) / (1 + np.linalg.norm(lp.c))
    assert rel_p <= 1e-6 * (1 + 1e-9) and rel_d <= 1e-6 * (1 + 1e-9), (rel_p, rel_d)
    assert abs(rel_p - rg["rel_primal_res"]) <= 1e-9 + 1e-6 * rel_p
    assert abs(rel_d - rg["rel_dual_res"]) <= 1e-9 + 1e-6 * rel_d


def test_infeasibility_no_rows(pdhg, oracle_lib):
    """m = 0: the primal ray alone certifies an unbounded objective."""
    _say("case: unbounded LP without constraint rows, n=40")
    n = 40
    c = np.random.default_rng(0).uniform(0.5, 2.0, n)
    c[7] = -1.0
    lp = gen.LP(0, n, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), c, np.zeros(0), np.zeros(0),
                np.zeros(n), np.full(n, np.inf))
    xo, _, ro = oracle_lib.Oracle(lp, iteration_limit=100000).solve()
    with pdhg.Solver.from_lp(lp, iteration_limit=100000) as s:
        xg, _, rg = s.solve()
    assert rg["status_name"] == ro["status_name"] == "dual_infeasible"
    assert rg["iterations"] == ro["iterations"]
    assert rel_inf(to_np(xg), xo) <= 1e-12
