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
    """The frozen map is piecewise linear in c (the projection patterns switch
    at kinks), so a difference quotient only matches the adjoint when no kink
    lies inside the step: each coordinate is checked with a central quotient
    (h = 1e-7) and the two one-sided ones (h = 1e-8), one of which must agree.
    A wrong adjoint fails all three."""
    _say("case: adjoint vs difference quotients through the frozen schedule")
    lps = _small_lps()[:3]
    T = 200
    rng = np.random.default_rng(7)
    with pdhg.BatchSolver.from_lps(lps) as bs:
        c0 = np.concatenate([lp.c for lp in lps])
        x, y = bs.unrolled(T)
        wx, wy = rng.standard_normal(bs.vec_n), rng.standard_normal(bs.vec_m)
        gc, _, _ = bs.backward(wx, wy)
        gc = to_np(gc)

        def loss(c):
            bs.update_data(c=c)
            xx, yy = bs.unrolled(T, replay=True)
            xx, yy = to_np(xx), to_np(yy)
            return np.array([wx[cs] @ xx[cs] + wy[rs] @ yy[rs]
                             for cs, rs in (bs.instance_slices(b) for b in range(bs.batch))])

        l0 = loss(c0)
        n_max = max(lp.n for lp in lps)
        checked = 0
        for j in range(0, n_max, 5):
            def unit(h):
                e = np.zeros(bs.vec_n)
                for b in range(bs.batch):
                    cs, _ = bs.instance_slices(b)
                    if j < cs.stop - cs.start:
                        e[cs.start + j] = h
                return e
            central = (loss(c0 + unit(1e-7)) - loss(c0 - unit(1e-7))) / 2e-7
            fwd = (loss(c0 + unit(1e-8)) - l0) / 1e-8
            bwd = (l0 - loss(c0 - unit(1e-8))) / 1e-8
            for b in range(bs.batch):
                cs, _ = bs.instance_slices(b)
                if j < cs.stop - cs.start:
                    g = gc[cs.start + j]
                    err = min(abs(central[b] - g), abs(fwd[b] - g), abs(bwd[b] - g))
                    assert err <= 2e-5 * (1 + abs(g)), (b, j, central[b], fwd[b], bwd[b], g)
                    checked += 1
        assert checked > 20
        bs.update_data(c=c0)


def test_envelope_gradients_at_convergence(pdhg, oracle_lib):
    """d(c'x*)/dc = x* and, on equality rows of a planted LP, d(c'x*)/db = y*.
    The second identity needs a unique dual solution; some planted instances
    are degenerate, so the seed is one whose three duals are unique (checked
    with the oracle's reverse pass)."""
    _say("case: envelope gradients, planted LPs")
    lps = gen.ragged_planted_batch(batch=3, m_lo=30, m_hi=40, density=0.15, seed=3904)
    # T past the oracle's iteration count at eps 1e-10 for every instance, so
    # the unrolled output sits at the solution
    T = max(oracle_lib.Oracle(lp, eps=1e-10).solve()[2]["iterations"] for lp in lps) + 200
    with pdhg.BatchSolver.from_lps(lps) as bs:
        x, y = bs.unrolled(T)
        c = np.concatenate([lp.c for lp in lps])
        gc, glc, guc = bs.backward(c)
        x, gc, glc, guc = to_np(x), to_np(gc), to_np(glc), to_np(guc)
        for b, lp in enumerate(lps):
            cs, rs = bs.instance_slices(b)
            xs, ys, r = oracle_lib.Oracle(lp, eps=1e-10).solve()
            grad_c = x[cs] + gc[cs]
            assert np.abs(grad_c - xs).max() <= 1e-6 * (1 + np.abs(xs).max())
            eq = np.isfinite(lp.lc) & (lp.lc == lp.uc)
            grad_b = glc[rs] + guc[rs]
            assert np.abs(grad_b[eq] - ys[eq]).max() <= 1e-6 * (1 + np.abs(ys[eq]).max())


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
