"""Pins of the oracle's loss heads (oracle/heads.py) against properties fixed
by their definitions: basis selection and linearity, the adjoint identity
between the cost model and its weight gradient, zero regret of the
shortest-path flow (Dijkstra) and non-negative regret of any other feasible
flow, and finite differences of the QP value. Also the composite gradient of
the regret through the unrolled solver against difference quotients."""

import numpy as np
import pytest

import gen
from oracle import heads


def test_linear_costs_basis_and_linearity():
    rng = np.random.default_rng(0)
    f = rng.standard_normal((3, 7, 4))
    for k in range(4):
        e = np.zeros(4); e[k] = 1.0
        np.testing.assert_array_equal(heads.linear_costs(f, e), f[:, :, k])
    W1, W2 = rng.standard_normal(4), rng.standard_normal(4)
    np.testing.assert_allclose(heads.linear_costs(f, 2 * W1 - 3 * W2),
                               2 * heads.linear_costs(f, W1) - 3 * heads.linear_costs(f, W2), atol=1e-13)


def test_weight_gradient_is_the_adjoint():
    """<gc, C(W)> = <C^T gc, W> for the linear map C(W) = f W."""
    rng = np.random.default_rng(1)
    f = rng.standard_normal((4, 11, 5))
    for _ in range(5):
        W, gc = rng.standard_normal(5), rng.standard_normal((4, 11))
        lhs = np.sum(gc * heads.linear_costs(f, W))
        rhs = np.dot(heads.linear_costs_backward(f, gc), W)
        assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))


def _path_flow(sb, b, costs):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra
    tails, heads_ = sb.meta["tails"], sb.meta["heads"]
    w = sp.csr_matrix((costs, (tails, heads_)), shape=(sb.m, sb.m))
    s, t = int(sb.meta["source"][b]), int(sb.meta["sink"][b])
    dist, pred = dijkstra(w, indices=s, return_predecessors=True)
    arc = {(int(u), int(v)): a for a, (u, v) in enumerate(zip(tails, heads_))}
    x = np.zeros(sb.n)
    v = t
    while v != s:
        u = int(pred[v])
        x[arc[(u, v)]] = sb.meta["supply"][b]
        v = u
    return x, sb.meta["supply"][b] * dist[t]


def test_regret_zero_at_shortest_path_and_nonnegative_elsewhere():
    sb, f, w_star, W0 = gen.shortest_path_learning(batch=3, rows=6, cols=6, seed=4100)
    rng = np.random.default_rng(2)
    for b in range(3):
        xs, vs = _path_flow(sb, b, sb.c[b])
        assert abs(heads.regret(sb.c[b:b + 1], xs[None], [vs])[0]) <= 1e-12 * (1 + vs)
        # the shortest path under perturbed costs is feasible, so its regret is >= 0
        xp, _ = _path_flow(sb, b, sb.c[b] * rng.uniform(0.5, 1.5, sb.n))
        assert heads.regret(sb.c[b:b + 1], xp[None], [vs])[0] >= -1e-12


def test_true_costs_follow_the_feature_model():
    sb, f, w_star, W0 = gen.shortest_path_learning(batch=2, rows=5, cols=5, seed=4101)
    z = heads.linear_costs(f, w_star)
    np.testing.assert_allclose(sb.c, 1 + 9 / (1 + np.exp(-z)), rtol=1e-14)
    assert sb.c.min() >= 1.0 and sb.c.max() <= 10.0


def test_qp_value_gradient_and_dense_form():
    p = gen.portfolio_qp_batch(batch=3, n=9, rank=2, seed=4200)
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 0.2, size=(3, 9))
    val, grad = heads.qp_value(p["F"], p["d"], p["c"], x)
    for b in range(3):
        Q = np.zeros((9, 9))
        for i in range(9):
            for j in range(9):
                Q[i, j] = sum(p["F"][i, k] * p["F"][j, k] for k in range(2)) + (p["d"][b, i] if i == j else 0.0)
        assert abs(val[b] - (0.5 * x[b] @ Q @ x[b] + p["c"][b] @ x[b])) <= 1e-14
        h = 1e-5
        for j in range(9):
            e = np.zeros(9); e[j] = h
            vp = heads.qp_value(p["F"], p["d"][b:b + 1], p["c"][b:b + 1], (x[b] + e)[None])[0][0]
            vm = heads.qp_value(p["F"], p["d"][b:b + 1], p["c"][b:b + 1], (x[b] - e)[None])[0][0]
            assert abs((vp - vm) / (2 * h) - grad[b, j]) <= 1e-8


def test_regret_weight_gradient_through_the_unrolled_solver(oracle_lib):
    """dL/dW for L(W) = sum_b regret(c_true, x_T(f W), v*) with x_T the frozen
    unrolled map: reverse pass with cotangent c_true, then the adjoint of the
    cost model; checked against difference quotients of the whole pipeline
    (kink-aware: central or one-sided must agree)."""
    sb, f, w_star, W = gen.shortest_path_learning(batch=2, rows=4, cols=4, seed=4102)
    W = W + 0.3          # costs well away from zero
    T = 120
    vstar = np.array([_path_flow(sb, b, sb.c[b])[1] for b in range(2)])

    def pipeline(Wv, sched=None):
        ch = heads.linear_costs(f, Wv)
        xs, scheds = [], []
        for b in range(2):
            lp = sb.instance(b)
            lp.c = ch[b]
            o = oracle_lib.Oracle(lp)
            if sched is None:
                x, _, sr, sw = o.unrolled(T)
            else:
                x, _, sr, sw = o.unrolled(T, *sched[b])
            xs.append(x)
            scheds.append((sr, sw))
        return np.array(xs), scheds

    x, scheds = pipeline(W)
    gcs = []
    for b in range(2):
        lp = sb.instance(b)
        lp.c = heads.linear_costs(f, W)[b]
        gc, _, _ = oracle_lib.Oracle(lp).backward(T, *scheds[b], sb.c[b], np.zeros(sb.m))
        gcs.append(gc)
    gW = heads.linear_costs_backward(f, np.array(gcs))

    def L(Wv):
        xx, _ = pipeline(Wv, scheds)
        return heads.regret(sb.c, xx, vstar).sum()

    L0 = L(W)
    for k in range(W.size):
        e = np.zeros(W.size)
        e[k] = 1.0
        central = (L(W + 1e-7 * e) - L(W - 1e-7 * e)) / 2e-7
        fwd = (L(W + 1e-8 * e) - L0) / 1e-8
        bwd = (L0 - L(W - 1e-8 * e)) / 1e-8
        err = min(abs(central - gW[k]), abs(fwd - gW[k]), abs(bwd - gW[k]))
        assert err <= 1e-5 * (1 + abs(gW[k])), (k, central, fwd, bwd, gW[k])


# ---- SPO+ and perturbed Fenchel-Young heads ------------------------------
# Exact optima of the small grid flows come from HiGHS (scipy), so these pins
# do not depend on the PDHG oracle.

def _exact(lp, costs):
    """Vertex optimum and value of min costs'x s.t. lc <= A x <= uc, lv <= x <= uv."""
    from scipy.optimize import linprog
    import scipy.sparse as sp
    A = sp.csr_matrix((lp.val, lp.colidx, lp.rowptr), shape=(lp.m, lp.n))
    eq = np.isfinite(lp.lc) & np.isfinite(lp.uc) & (lp.lc == lp.uc)
    ub_rows, ub_rhs = [], []
    for i in np.where(~eq)[0]:
        if np.isfinite(lp.uc[i]):
            ub_rows.append(A[i]); ub_rhs.append(lp.uc[i])
        if np.isfinite(lp.lc[i]):
            ub_rows.append(-A[i]); ub_rhs.append(-lp.lc[i])
    kw = {}
    if eq.any():
        kw.update(A_eq=A[eq], b_eq=lp.lc[eq])
    if ub_rows:
        kw.update(A_ub=sp.vstack(ub_rows), b_ub=np.array(ub_rhs))
    bounds = [(None if not np.isfinite(l) else l, None if not np.isfinite(u) else u)
              for l, u in zip(lp.lv, lp.uv)]
    r = linprog(costs, bounds=bounds, method="highs", **kw)
    assert r.status == 0, r.message
    return r.x, r.fun


def _spo_case(seed, B=3, rows=4, cols=4):
    sb, f, w_true, W0 = gen.shortest_path_learning(batch=B, rows=rows, cols=cols, seed=seed)
    rng = np.random.default_rng(seed)
    c_hat = heads.linear_costs(f, W0 + rng.normal(0, 1, W0.shape))
    return sb, c_hat


def _spo_eval(sb, c_hat):
    B = c_hat.shape[0]
    ws, zs, wt = [], [], []
    for b in range(B):
        lp = sb.instance(b)
        w, z = _exact(lp, sb.c[b])
        ws.append(w); zs.append(z)
        wt.append(_exact(lp, heads.spo_plus_costs(c_hat[b:b + 1], sb.c[b:b + 1])[0])[0])
    return heads.spo_plus(c_hat, sb.c, np.array(ws), np.array(zs), np.array(wt)), np.array(ws), np.array(zs)


def test_spo_plus_closed_form_on_the_simplex():
    """min c'w over the probability simplex picks the cheapest coordinate, so
    SPO+ = max_i (c - 2 c_hat)_i + 2 c_hat_{i*} - c_{i*} with i* = argmin c."""
    c = np.array([[3.0, 1.0, 2.0]])
    c_hat = np.array([[0.5, 2.0, 1.0]])
    w_star = np.array([[0.0, 1.0, 0.0]]); z_star = np.array([1.0])
    inner = heads.spo_plus_costs(c_hat, c)           # [-2, 3, 0]: w_tilde = e_0
    np.testing.assert_array_equal(inner, [[-2.0, 3.0, 0.0]])
    loss, grad = heads.spo_plus(c_hat, c, w_star, z_star, np.array([[1.0, 0.0, 0.0]]))
    # max_i (c - 2 c_hat)_i = max(2, -3, 0) = 2; + 2*2.0 - 1.0 = 5
    assert loss[0] == 5.0
    np.testing.assert_array_equal(grad, [[-2.0, 2.0, 0.0]])


def test_spo_plus_zero_at_true_costs_and_above_regret():
    """SPO+(c, c) = 0, and SPO+(c_hat, c) >= regret(c_hat, c) = c'w*(c_hat) - z*(c) >= 0."""
    sb, c_hat = _spo_case(4500)
    (loss0, grad0), ws, zs = _spo_eval(sb, sb.c.copy())
    scale = np.abs(zs) + 1.0
    assert np.all(np.abs(loss0) <= 1e-9 * scale), loss0
    assert np.abs(grad0).max() <= 1e-7
    (loss, grad), ws, zs = _spo_eval(sb, c_hat)
    for b in range(c_hat.shape[0]):
        w_hat, _ = _exact(sb.instance(b), c_hat[b])
        reg = np.dot(sb.c[b], w_hat) - zs[b]
        assert reg >= -1e-9 * scale[b]
        assert loss[b] >= reg - 1e-9 * scale[b], (b, loss[b], reg)


def test_spo_plus_subgradient_inequality_and_directional_derivative():
    """The loss is convex in c_hat with subgradient 2 (w* - w_tilde):
    loss(c') >= loss(c_hat) + grad'(c' - c_hat) for any c', and where the
    inner optimum does not move the loss is affine with exactly that slope."""
    sb, c_hat = _spo_case(4501)
    rng = np.random.default_rng(9)
    (loss, grad), _, _ = _spo_eval(sb, c_hat)
    for _ in range(4):
        c2 = c_hat + rng.normal(0, 1.0, c_hat.shape)
        (loss2, _), _, _ = _spo_eval(sb, c2)
        lin = loss + np.sum(grad * (c2 - c_hat), axis=1)
        assert np.all(loss2 >= lin - 1e-8 * (1 + np.abs(loss))), (loss2, lin)
    d = rng.normal(0, 1.0, c_hat.shape)
    h = 1e-6
    (lp_, _), _, _ = _spo_eval(sb, c_hat + h * d)
    (lm_, _), _, _ = _spo_eval(sb, c_hat - h * d)
    slope = np.sum(grad * d, axis=1)
    np.testing.assert_allclose((lp_ - lm_) / (2 * h), slope, rtol=1e-5, atol=1e-5)


def test_pfy_zero_noise_and_directional_derivative():
    """With eps = 0 every sample is the optimum under c_hat: at c_hat = c the
    loss and gradient vanish. With fixed draws the sampled loss is piecewise
    affine in c_hat with slope w* - mean_m w_m."""
    sb, c_hat = _spo_case(4502, B=2)
    B, n = c_hat.shape
    M = 3
    rng = np.random.default_rng(5)
    Z = rng.standard_normal((B, M, n))
    ws = np.array([_exact(sb.instance(b), sb.c[b])[0] for b in range(B)])

    def samples(ch, eps):
        pc = heads.pfy_costs(ch, Z, eps)
        assert pc.shape == (B, M, n)
        return np.array([[_exact(sb.instance(b), pc[b, m])[0] for m in range(M)] for b in range(B)])

    loss0, grad0 = heads.pfy(sb.c, ws, Z, 0.0, samples(sb.c, 0.0))
    assert np.abs(loss0).max() <= 1e-9 * (1 + np.abs(sb.c).sum())
    assert np.abs(grad0).max() <= 1e-7
    eps = 0.5
    loss, grad = heads.pfy(c_hat, ws, Z, eps, samples(c_hat, eps))
    d = rng.normal(0, 1.0, c_hat.shape)
    h = 1e-6
    lp_, _ = heads.pfy(c_hat + h * d, ws, Z, eps, samples(c_hat + h * d, eps))
    lm_, _ = heads.pfy(c_hat - h * d, ws, Z, eps, samples(c_hat - h * d, eps))
    np.testing.assert_allclose((lp_ - lm_) / (2 * h), np.sum(grad * d, axis=1), rtol=1e-5, atol=1e-5)
    # the gradient averages the samples in order: one sample reproduces w* - w_1
    l1, g1 = heads.pfy(c_hat, ws, Z[:, :1], eps, samples(c_hat, eps)[:, :1])
    s1 = samples(c_hat, eps)[:, 0]
    np.testing.assert_allclose(g1, ws - s1, atol=1e-12)


def test_pfy_closed_form_on_the_simplex():
    """Simplex in R^3, c_hat = (1, 2, 3), w* = e_0, eps = 1 and two draws:
    Z_1 = (2, 0, 0) gives costs (3, 2, 3), optimum e_1 (value 2);
    Z_2 = (0, 0, -2.5) gives costs (1, 2, 0.5), optimum e_2 (value 0.5).
    loss = c_hat'w* - (2 + 0.5)/2 = -0.25, grad = e_0 - (e_1 + e_2)/2."""
    c_hat = np.array([[1.0, 2.0, 3.0]])
    Z = np.array([[[2.0, 0.0, 0.0], [0.0, 0.0, -2.5]]])
    np.testing.assert_array_equal(heads.pfy_costs(c_hat, Z, 1.0), [[[3.0, 2.0, 3.0], [1.0, 2.0, 0.5]]])
    w_star = np.array([[1.0, 0.0, 0.0]])
    ws = np.array([[[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]])
    loss, grad = heads.pfy(c_hat, w_star, Z, 1.0, ws)
    assert loss[0] == -0.25
    np.testing.assert_array_equal(grad, [[1.0, -0.5, -0.5]])
