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
