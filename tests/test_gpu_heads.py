"""GPU parity of the loss heads (pdhg_linear_costs, pdhg_regret,
pdhg_linear_costs_backward, pdhg_qp_value) and of the whole learning step
(cost model -> unrolled batch -> regret -> reverse pass -> weight gradient)
against the oracle."""

import sys

import numpy as np
import pytest

import gen
from gpu_util import rel_inf, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_09734_amd.heads as h
    import paper_2412_09734_amd.solver as s
    return h, s


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_heads_match_oracle(mods):
    from oracle import heads as oh
    h, _ = mods
    _say("case: loss heads vs oracle, B=5 n=37 p=5; QP B=4 n=300 r=7")
    rng = np.random.default_rng(11)
    f = rng.standard_normal((5, 37, 5))
    W = rng.standard_normal(5)
    assert rel_inf(to_np(h.linear_costs(f, W)), oh.linear_costs(f, W)) <= 1e-13
    ct, x, vs = rng.uniform(1, 10, (5, 37)), rng.uniform(0, 1, (5, 37)), rng.standard_normal(5)
    assert rel_inf(to_np(h.regret(ct, x, vs)), oh.regret(ct, x, vs)) <= 1e-12
    gc = rng.standard_normal((5, 37))
    assert rel_inf(to_np(h.linear_costs_backward(f, gc)), oh.linear_costs_backward(f, gc)) <= 1e-12
    p = gen.portfolio_qp_batch(batch=4, n=300, rank=7, seed=4300)
    xq = rng.uniform(0, 0.1, (4, 300))
    val, grad = h.qp_value(p["F"], p["d"], p["c"], xq)
    vo, go = oh.qp_value(p["F"], p["d"], p["c"], xq)
    assert rel_inf(to_np(val), vo) <= 1e-12
    assert rel_inf(to_np(grad), go) <= 1e-12
    val2, none = h.qp_value(p["F"], p["d"], p["c"], xq, grad=False)
    assert none is None and rel_inf(to_np(val2), vo) <= 1e-12


def test_heads_reject_bad_sizes(mods):
    import ctypes as C
    from paper_2412_09734_amd import _capi as capi
    _say("case: loss-head argument errors")
    L = capi.lib()
    assert L.pdhg_linear_costs(1, 4, 0, None, None, None, None) == -1
    assert L.pdhg_linear_costs(1, 4, 65, None, None, None, None) == -1
    assert L.pdhg_regret(2, 3, None, None, None, None, None) == -1
    assert L.pdhg_qp_value(1, 3, 33, None, None, None, None, None, None, None) == -1


def test_learning_step_matches_oracle(mods, oracle_lib):
    from oracle import heads as oh
    h, s = mods
    _say("case: learning step (costs -> unrolled T=150 -> regret -> reverse -> dW), 4 grids 6x6")
    sb, f, w_star, W = gen.shortest_path_learning(batch=4, rows=6, cols=6, seed=4400)
    W = W + 0.3
    T = 150
    vstar = np.array([oracle_lib.Oracle(sb.instance(b), eps=1e-10).solve()[2]["primal_obj"]
                      for b in range(4)])
    chat = h.linear_costs(f, W)
    with s.BatchSolver.from_shared(sb) as bs:
        bs.update_data(c=chat)
        x, _ = bs.unrolled(T)
        loss = h.regret(sb.c, x, vstar)
        gc = bs.backward(sb.c)[0]
        gW = h.linear_costs_backward(f, gc)
    ch = oh.linear_costs(f, W)
    xs, gcs = [], []
    for b in range(4):
        lp = sb.instance(b)
        lp.c = ch[b]
        o = oracle_lib.Oracle(lp)
        xo, _, sr, sw = o.unrolled(T)
        xs.append(xo)
        gcs.append(o.backward(T, sr, sw, sb.c[b], np.zeros(sb.m))[0])
    assert rel_inf(to_np(x), np.array(xs)) <= 1e-10
    assert rel_inf(to_np(loss), oh.regret(sb.c, np.array(xs), vstar)) <= 1e-9
    assert rel_inf(to_np(gW), oh.linear_costs_backward(f, np.array(gcs))) <= 1e-9


def test_surrogate_heads_match_oracle(mods):
    """SPO+ and perturbed Fenchel-Young heads on random inputs: the cost maps
    and gradients round exactly as the oracle's; the losses sum in another
    order (bound: a few ulps of the sum of absolute terms)."""
    from oracle import heads as oh
    h, _ = mods
    _say("case: SPO+ / PFY heads vs oracle, B=5 n=301, M=3")
    rng = np.random.default_rng(12)
    B, n, M = 5, 301, 3
    ch, ct = rng.standard_normal((B, n)), rng.uniform(1, 10, (B, n))
    ws, wt = rng.uniform(0, 1, (B, n)), rng.uniform(0, 1, (B, n))
    zs = rng.standard_normal(B)
    np.testing.assert_array_equal(to_np(h.spo_plus_costs(ch, ct)), oh.spo_plus_costs(ch, ct))
    loss, grad = h.spo_plus(ch, ct, ws, zs, wt)
    lo, go = oh.spo_plus(ch, ct, ws, zs, wt)
    np.testing.assert_array_equal(to_np(grad), go)
    scale = np.sum(np.abs(2 * ch * ws) + np.abs((2 * ch - ct) * wt), axis=1) + np.abs(zs)
    assert np.all(np.abs(to_np(loss) - lo) <= 1e-14 * n * scale)
    Z = rng.standard_normal((B, M, n))
    np.testing.assert_array_equal(to_np(h.pfy_costs(ch, Z, 0.3)), oh.pfy_costs(ch, Z, 0.3))
    wm = rng.uniform(0, 1, (B, M, n))
    loss, grad = h.pfy(ch, ws, Z, 0.3, wm)
    lo, go = oh.pfy(ch, ws, Z, 0.3, wm)
    np.testing.assert_array_equal(to_np(grad), go)
    scale = np.sum(np.abs(ch * ws), axis=1) + np.sum(np.abs((ch[:, None] + 0.3 * Z) * wm), axis=(1, 2)) / M
    assert np.all(np.abs(to_np(loss) - lo) <= 1e-14 * n * scale)


def test_surrogate_heads_reject_bad_input(mods):
    from paper_2412_09734_amd import _capi as capi
    _say("case: surrogate-head argument errors")
    L = capi.lib()
    assert L.pdhg_spo_plus_costs(-1, 3, None, None, None, None) == -1
    assert L.pdhg_spo_plus(2, 3, None, None, None, None, None, None, None, None) == -1
    assert L.pdhg_pfy_costs(1, 0, 3, None, None, 0.1, None, None) == -1
    assert L.pdhg_pfy_costs(1, 2, 0, None, None, float("nan"), None, None) == -1
    assert L.pdhg_pfy(1, 0, 3, None, None, None, 0.1, None, None, None, None) == -1


def _true_solutions(oracle_lib, sb, B):
    ws, zs = [], []
    for b in range(B):
        xo, _, ro = oracle_lib.Oracle(sb.instance(b), eps=1e-10).solve()
        ws.append(xo); zs.append(ro["primal_obj"])
    return np.array(ws), np.array(zs)


def test_spo_plus_step_matches_oracle(mods, oracle_lib):
    """cost model -> SPO+ costs -> batched solve (warm-started the second time)
    -> SPO+ loss and subgradient -> weight gradient, against the oracle's
    solves of the same inner problems."""
    from oracle import heads as oh
    h, s = mods
    _say("case: SPO+ learning step, 4 grids 6x6, inner solves to 1e-8")
    B = 4
    sb, f, w_true, W = gen.shortest_path_learning(batch=B, rows=6, cols=6, seed=4600)
    ws, zs = _true_solutions(oracle_lib, sb, B)
    chat = h.linear_costs(f, W)
    with s.BatchSolver.from_shared(sb, eps=1e-8) as bs:
        bs.update_data(c=h.spo_plus_costs(chat, sb.c))
        wt, _, res = bs.solve()
        loss, g = h.spo_plus(chat, sb.c, ws, zs, wt)
        gW = h.linear_costs_backward(f, g)
        wt2, _, res2 = bs.solve(x_init=wt)
        assert all(r["status_name"] == "optimal" for r in res + res2)
        assert sum(r["iterations"] for r in res2) < sum(r["iterations"] for r in res)
    ch = oh.linear_costs(f, W)
    inner = oh.spo_plus_costs(ch, sb.c)
    wto = []
    for b in range(B):
        lp = sb.instance(b)
        lp.c = inner[b]
        xo, _, ro = oracle_lib.Oracle(lp, eps=1e-8).solve()
        assert ro["iterations"] == res[b]["iterations"], (b, ro["iterations"], res[b]["iterations"])
        wto.append(xo)
    lo, go = oh.spo_plus(ch, sb.c, ws, zs, np.array(wto))
    # both sides solve to relative KKT 1e-8
    assert rel_inf(to_np(wt), np.array(wto)) <= 1e-6
    assert rel_inf(to_np(loss), lo) <= 1e-6
    assert rel_inf(to_np(gW), oh.linear_costs_backward(f, go)) <= 1e-6


def test_pfy_step_matches_oracle(mods, oracle_lib):
    """perturbed costs for B x M samples -> one batched solve of all samples ->
    Fenchel-Young loss and gradient, against the oracle."""
    from types import SimpleNamespace
    from oracle import heads as oh
    h, s = mods
    B, M, eps = 2, 3, 0.5
    _say(f"case: perturbed Fenchel-Young step, {B} grids 6x6, M={M} samples, inner solves to 1e-8")
    sb, f, w_true, W = gen.shortest_path_learning(batch=B, rows=6, cols=6, seed=4700)
    ws, zs = _true_solutions(oracle_lib, sb, B)
    Z = np.random.default_rng(8).standard_normal((B, M, sb.n))
    chat = h.linear_costs(f, W)
    pc = h.pfy_costs(chat, Z, eps)
    rep = lambda a: np.repeat(a, M, axis=0)
    samples = SimpleNamespace(m=sb.m, n=sb.n, rowptr=sb.rowptr, colidx=sb.colidx, val=sb.val,
                              c=pc.reshape(B * M, sb.n), lc=rep(sb.lc), uc=rep(sb.uc), lv=rep(sb.lv),
                              uv=rep(sb.uv))
    with s.BatchSolver.from_shared(samples, eps=1e-8) as bs:
        wm, _, res = bs.solve()
        assert all(r["status_name"] == "optimal" for r in res)
        loss, g = h.pfy(chat, ws, Z, eps, wm.reshape(B, M, sb.n))
    ch = oh.linear_costs(f, W)
    pco = oh.pfy_costs(ch, Z, eps)
    wmo = np.zeros((B, M, sb.n))
    for b in range(B):
        for m in range(M):
            lp = sb.instance(b)
            lp.c = pco[b, m]
            wmo[b, m] = oracle_lib.Oracle(lp, eps=1e-8).solve()[0]
    lo, go = oh.pfy(ch, ws, Z, eps, wmo)
    assert rel_inf(to_np(wm).reshape(B, M, sb.n), wmo) <= 1e-6
    assert rel_inf(to_np(loss), lo) <= 1e-6
    assert rel_inf(to_np(g), go) <= 1e-6
