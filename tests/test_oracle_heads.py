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
