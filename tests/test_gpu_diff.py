"""GPU parity of the unrolled forward and its adjoint (LP batches) against the
CPU oracle, central finite differences and the envelope closed forms."""

import sys

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


def _small_lps():
    lps = gen.ragged_planted_batch(batch=6, m_lo=20, m_hi=45, density=0.15, seed=3800)
    for i, lp in enumerate(lps):          # give some variables finite upper bounds
        lp.uv = lp.uv.copy()
        lp.uv[:: 3 + i] = 2.0
    return lps


def test_unrolled_forward_and_backward_match_oracle(pdhg, oracle_lib):
    _say("case: unrolled forward / adjoint vs oracle, ragged batch, T=300")
    lps = _small_lps()
    T = 300
    rng = np.random.default_rng(5)
    with pdhg.BatchSolver.from_lps(lps) as bs:
        x, y = bs.unrolled(T)
        gx = rng.standard_normal(bs.vec_n)
        gy = rng.standard_normal(bs.vec_m)
        gc, glc, guc = bs.backward(gx, gy)
        for b, lp in enumerate(lps):
            cs, rs = bs.instance_slices(b)
            o = oracle_lib.Oracle(lp)
            xo, yo, sr, sw = o.unrolled(T)
            assert rel_inf(to_np(x[cs]), xo) <= 1e-10, (b, rel_inf(to_np(x[cs]), xo))
            assert rel_inf(to_np(y[rs]), yo) <= 1e-10
            gco, glco, guco = o.backward(T, sr, sw, gx[cs], gy[rs])
            assert rel_inf(to_np(gc[cs]), gco) <= 1e-9, (b, rel_inf(to_np(gc[cs]), gco))
            assert rel_inf(to_np(glc[rs]), glco) <= 1e-9
            assert rel_inf(to_np(guc[rs]), guco) <= 1e-9


def test_adjoint_matches_finite_differences(pdhg):
    _say("case: adjoint vs central differences (h=1e-6) through the frozen schedule")
    lps = _small_lps()[:3]
    T = 200
    rng = np.random.default_rng(7)
    with pdhg.BatchSolver.from_lps(lps) as bs:
        c0 = np.concatenate([lp.c for lp in lps])
        x, y = bs.unrolled(T)
        wx, wy = rng.standard_normal(bs.vec_n), rng.standard_normal(bs.vec_m)
        gc, _, _ = bs.backward(wx, wy)
        gc = to_np(gc)
        h = 1e-6

        def loss(c):
            bs.update_data(c=c)
            xx, yy = bs.unrolled(T, replay=True)
            xx, yy = to_np(xx), to_np(yy)
            return np.array([wx[cs] @ xx[cs] + wy[rs] @ yy[rs]
                             for cs, rs in (bs.instance_slices(b) for b in range(bs.batch))])

        n_max = max(lp.n for lp in lps)
        for j in range(0, n_max, 7):
            e = np.zeros(bs.vec_n)
            for b in range(bs.batch):
                cs, _ = bs.instance_slices(b)
                if j < cs.stop - cs.start:
                    e[cs.start + j] = h
            fd = (loss(c0 + e) - loss(c0 - e)) / (2 * h)
            for b in range(bs.batch):
                cs, _ = bs.instance_slices(b)
                if j < cs.stop - cs.start:
                    g = gc[cs.start + j]
                    assert abs(fd[b] - g) <= 1e-6 * (1 + abs(fd[b])), (b, j, fd[b], g)
        bs.update_data(c=c0)


def test_envelope_gradients_at_convergence(pdhg, oracle_lib):
    """d(c'x*)/dc = x* and, on equality rows of a planted LP, d(c'x*)/db = y*."""
    _say("case: envelope gradients, planted LPs")
    lps = gen.ragged_planted_batch(batch=3, m_lo=30, m_hi=40, density=0.15, seed=3900)
    T = 4000
    with pdhg.BatchSolver.from_lps(lps) as bs:
        x, y = bs.unrolled(T)
        c = np.concatenate([lp.c for lp in lps])
        gc, glc, guc = bs.backward(c)
        x, gc, glc, guc = to_np(x), to_np(gc), to_np(glc), to_np(guc)
        for b, lp in enumerate(lps):
            cs, rs = bs.instance_slices(b)
            xs, ys, r = oracle_lib.Oracle(lp, eps=1e-10).solve()
            grad_c = x[cs] + gc[cs]
            assert np.abs(grad_c - xs).max() <= 2e-3 * (1 + np.abs(xs).max())
            eq = np.isfinite(lp.lc) & (lp.lc == lp.uc)
            grad_b = glc[rs] + guc[rs]
            assert np.abs(grad_b[eq] - ys[eq]).max() <= 2e-3 * (1 + np.abs(ys[eq]).max())


def test_autograd_function(pdhg):
    import torch
    _say("case: torch.autograd.Function over the unrolled batch")
    sb = gen.grid_mincost_batch(batch=4, rows=6, cols=6, seed=3300)
    with pdhg.BatchSolver.from_shared(sb) as bs:
        c = torch.tensor(sb.c, dtype=torch.float64, device="cuda", requires_grad=True)
        x = pdhg.UnrolledLP.apply(c, bs, 150)
        w = torch.randn_like(x)
        (x * w).sum().backward()
        gc, _, _ = bs.backward(w)
        assert torch.equal(c.grad, gc)
