"""Problem generators.

All matrices are CSR with int32 indices, strictly increasing column indices
inside a row and float64 values; absent bounds are +-inf.

Workload recipes (the paper's instances are not available, these stand in for
them with the same shapes and structure):

* planted sparse LP: pattern, values, then a planted optimal primal-dual pair
  (x*, y*) so that the optimal value V* = sum_eq y*_i b_i is known exactly;
* large Zipf LP: column degrees follow a truncated power law (mean 10), rows
  are scaled by LogUniform(1e-2, 1e2);
* dense planted LP: i.i.d. N(0, 1), all rows equalities;
* grid min-cost flow: node-arc incidence of a directed 4-neighbour grid;
* ragged batch: planted sparse LPs of uneven size;
* portfolio QP: Q = F F' + diag(d), sum(x) = 1, 0 <= x <= 0.1.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

INF = np.inf


def seed_for(cfg: int, instance: int = 0) -> int:
    """Seed convention: 1000 * workload id + instance index."""
    return 1000 * int(cfg) + int(instance)


@dataclass
class LP:
    """One problem instance (LP when q_kind == 'none')."""

    m: int
    n: int
    rowptr: Optional[np.ndarray]  # int32 [m+1] (None when dense)
    colidx: Optional[np.ndarray]  # int32 [nnz]
    val: Optional[np.ndarray]  # float64 [nnz]
    c: np.ndarray
    lc: np.ndarray
    uc: np.ndarray
    lv: np.ndarray
    uv: np.ndarray
    dense: Optional[np.ndarray] = None  # float64 [m, n] row-major (dense format)
    # quadratic term
    q_kind: str = "none"  # 'none' | 'csr' | 'lowrank'
    q_rowptr: Optional[np.ndarray] = None
    q_colidx: Optional[np.ndarray] = None
    q_val: Optional[np.ndarray] = None
    q_factor: Optional[np.ndarray] = None  # [n, r] row-major
    q_diag: Optional[np.ndarray] = None  # [n]
    # planted data (when known)
    x_star: Optional[np.ndarray] = None
    y_star: Optional[np.ndarray] = None
    v_star: Optional[float] = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        if self.dense is not None:
            return self.m * self.n
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        if self.dense is not None:
            return self.dense
        return dense_from_csr(self.m, self.n, self.rowptr, self.colidx, self.val)

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """A @ x (problem construction helper, float64)."""
        if self.dense is not None:
            return self.dense @ x
        return _csr_matvec(self.m, self.rowptr, self.colidx, self.val, x)

    def rmatvec(self, y: np.ndarray) -> np.ndarray:
        """A.T @ y (problem construction helper, float64)."""
        if self.dense is not None:
            return self.dense.T @ y
        return _csr_rmatvec(self.n, self.rowptr, self.colidx, self.val, y)


@dataclass
class SharedBatch:
    """B instances sharing one constraint matrix; vectors are [B, n] / [B, m]."""

    m: int
    n: int
    rowptr: np.ndarray
    colidx: np.ndarray
    val: np.ndarray
    c: np.ndarray
    lc: np.ndarray
    uc: np.ndarray
    lv: np.ndarray
    uv: np.ndarray
    v_star: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)
    q_factor: Optional[np.ndarray] = None   # QP batches: F [n, r] shared,
    q_diag: Optional[np.ndarray] = None     # d [B, n]: Q_b = F F' + diag(d_b)

    @property
    def batch(self) -> int:
        return int(self.c.shape[0])

    def instance(self, b: int) -> LP:
        q = {}
        if self.q_factor is not None:
            q = dict(q_kind="lowrank", q_factor=self.q_factor, q_diag=self.q_diag[b].copy())
        return LP(self.m, self.n, self.rowptr, self.colidx, self.val,
                  self.c[b].copy(), self.lc[b].copy(), self.uc[b].copy(),
                  self.lv[b].copy(), self.uv[b].copy(),
                  v_star=None if self.v_star is None else float(self.v_star[b]),
                  meta={k: (v[b] if isinstance(v, np.ndarray) and v.ndim >= 1
                            and v.shape[0] == self.batch else v)
                        for k, v in self.meta.items()}, **q)


# ----------------------------------------------------------------------------
# CSR helpers (construction only)


def _csr_matvec(m, rowptr, colidx, val, x):
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    out = np.zeros(m)
    np.add.at(out, rows, val * x[colidx])
    return out


def _csr_rmatvec(n, rowptr, colidx, val, y):
    m = len(rowptr) - 1
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    out = np.zeros(n)
    np.add.at(out, colidx, val * y[rows])
    return out


def csr_from_dense(a: np.ndarray):
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    mask = a != 0.0
    counts = mask.sum(axis=1)
    rowptr = np.zeros(m + 1, dtype=np.int32)
    np.cumsum(counts, out=rowptr[1:])
    r, cidx = np.nonzero(mask)
    return rowptr, cidx.astype(np.int32), a[r, cidx].astype(np.float64)


def dense_from_csr(m, n, rowptr, colidx, val):
    out = np.zeros((m, n))
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    out[rows, colidx] = val
    return out


def _csr_from_keys(m: int, n: int, rows: np.ndarray, cols: np.ndarray):
    """Sorted, de-duplicated CSR pattern from coordinate lists."""
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    key = np.unique(key)
    r = (key // n).astype(np.int64)
    cidx = (key % n).astype(np.int32)
    counts = np.bincount(r, minlength=m)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    assert rowptr[-1] < 2**31
    return rowptr.astype(np.int32), cidx, r


# ----------------------------------------------------------------------------
# planted optimum


def _plant(rng, m, n, matvec, rmatvec, rho, eq_frac, eq_all=False):
    """Planted optimal pair for min c'x, rows = / <= / >=, x >= 0.

    Support of x*: exactly round(rho n) columns, values U(0,1).
    Equality rows: round(eq_frac m) rows (all when eq_all), y*_i ~ N(0,1).
    Other rows: y*_i = 0, slack U(0,1), '<=' or '>=' with probability 1/2.
    Reduced costs: 0 on the support, U(0,1) off it; c = A'y* + s.
    """
    x_star = np.zeros(n)
    ns = int(round(rho * n))
    supp = rng.choice(n, size=ns, replace=False)
    x_star[supp] = rng.random(ns)
    ax = matvec(x_star)
    y_star = np.zeros(m)
    if eq_all:
        eq = np.arange(m)
    else:
        eq = np.sort(rng.choice(m, size=int(round(eq_frac * m)), replace=False))
    y_star[eq] = rng.standard_normal(len(eq))
    lc = np.full(m, -INF)
    uc = np.full(m, INF)
    lc[eq] = ax[eq]
    uc[eq] = ax[eq]
    is_eq = np.zeros(m, dtype=bool)
    is_eq[eq] = True
    ineq = np.nonzero(~is_eq)[0]
    slack = rng.random(len(ineq))
    le = rng.random(len(ineq)) < 0.5
    uc[ineq[le]] = ax[ineq[le]] + slack[le]
    lc[ineq[~le]] = ax[ineq[~le]] - slack[~le]
    s = rng.random(n)
    s[supp] = 0.0
    c = rmatvec(y_star) + s
    v_star = float(np.dot(y_star[eq], ax[eq]))
    return c, lc, uc, x_star, y_star, v_star


def planted_sparse_lp(m: int = 200, n: int = 400, density: float = 0.02,
                      rho: float = 0.5, eq_frac: float = 0.6,
                      seed: int = 0) -> LP:
    """Planted sparse LP: Bernoulli(density) pattern, N(0,1) values, x >= 0.

    With the defaults this is the small single-LP workload
    (m=200, n=400, ~2% density)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    r, cidx = np.nonzero(mask)
    rowptr = np.zeros(m + 1, dtype=np.int32)
    np.cumsum(mask.sum(axis=1), out=rowptr[1:])
    colidx = cidx.astype(np.int32)
    val = rng.standard_normal(len(colidx))
    mv = lambda x: _csr_matvec(m, rowptr, colidx, val, x)  # noqa: E731
    rmv = lambda y: _csr_rmatvec(n, rowptr, colidx, val, y)  # noqa: E731
    c, lc, uc, xs, ys, vs = _plant(rng, m, n, mv, rmv, rho, eq_frac)
    return LP(m, n, rowptr, colidx, val, c, lc, uc, np.zeros(n), np.full(n, INF),
              x_star=xs, y_star=ys, v_star=vs,
              meta=dict(kind="planted_sparse", seed=seed, density=density))


def zipf_pmf(kmax: int = 2000, s: float = 1.7948) -> np.ndarray:
    k = np.arange(1, kmax + 1, dtype=np.float64)
    p = k ** (-s)
    return p / p.sum()


def large_zipf_lp(m: int = 1_000_000, n: int = 2_000_000, kmax: int = 2000,
                  s: float = 1.7948, rho: float = 0.5, eq_frac: float = 0.6,
                  box_frac: float = 0.5, box_upper: float = 10.0,
                  seed: int = 1000) -> LP:
    """Large sparse planted LP with Zipf column degrees (mean ~10, max kmax).

    Row indices are uniform per column (duplicates dropped); values are
    N(0,1) times a per-row factor 10^U(-2, 2). Half of the columns get the
    upper bound box_upper. With the defaults: m=1e6, n=2e6, nnz ~ 2e7."""
    rng = np.random.default_rng(seed)
    pmf = zipf_pmf(kmax, s)
    deg = rng.choice(np.arange(1, kmax + 1, dtype=np.int64), size=n, p=pmf)
    deg = np.minimum(deg, m)
    cols = np.repeat(np.arange(n, dtype=np.int32), deg)
    rows = rng.integers(0, m, size=len(cols), dtype=np.int64)
    rowptr, colidx, rr = _csr_from_keys(m, n, rows, cols)
    del cols, rows
    row_scale = 10.0 ** rng.uniform(-2.0, 2.0, size=m)
    val = rng.standard_normal(len(colidx)) * row_scale[rr]
    del rr
    try:
        import scipy.sparse as sp
        a = sp.csr_matrix((val, colidx, rowptr), shape=(m, n))
        mv = lambda x: a @ x  # noqa: E731
        at = a.T.tocsr()
        rmv = lambda y: at @ y  # noqa: E731
    except ImportError:  # pragma: no cover
        mv = lambda x: _csr_matvec(m, rowptr, colidx, val, x)  # noqa: E731
        rmv = lambda y: _csr_rmatvec(n, rowptr, colidx, val, y)  # noqa: E731
    c, lc, uc, xs, ys, vs = _plant(rng, m, n, mv, rmv, rho, eq_frac)
    uv = np.full(n, INF)
    boxed = rng.choice(n, size=int(round(box_frac * n)), replace=False)
    uv[boxed] = box_upper
    return LP(m, n, rowptr, colidx, val, c, lc, uc, np.zeros(n), uv,
              x_star=xs, y_star=ys, v_star=vs,
              meta=dict(kind="large_zipf", seed=seed))


def dense_planted_lp(m: int = 20_000, n: int = 40_000, rho: float = 0.3,
                     seed: int = 2000) -> LP:
    """Dense planted LP, i.i.d. N(0,1) row-major, all rows equalities, x >= 0."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n))
    c, lc, uc, xs, ys, vs = _plant(rng, m, n, lambda x: a @ x, lambda y: a.T @ y,
                                   rho, 1.0, eq_all=True)
    return LP(m, n, None, None, None, c, lc, uc, np.zeros(n), np.full(n, INF),
              dense=a, x_star=xs, y_star=ys, v_star=vs,
              meta=dict(kind="dense_planted", seed=seed))


def dense_knapsack_lp(d: int = 1_000, items: int = 100_000, seed: int = 2500) -> LP:
    """LP relaxation of a multi-dimensional knapsack (the dense instance shape
    of the paper's hardware comparison): weights W ~ U(0,1) [d, items]
    row-major, item values v ~ U(0,1), capacities b = 1/4 of each row's total
    weight, 0 <= x <= 1. Stated as min (-v)'x s.t. W x <= b (value
    maximisation)."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.0, 1.0, size=(d, items))
    v = rng.uniform(0.0, 1.0, size=items)
    b = 0.25 * w.sum(axis=1)
    return LP(d, items, None, None, None, -v, np.full(d, -INF), b, np.zeros(items),
              np.ones(items), dense=w, meta=dict(kind="dense_knapsack", seed=seed))


# ----------------------------------------------------------------------------
# grid min-cost flow (node-arc incidence, out - in)


def grid_incidence(rows: int = 32, cols: int = 32):
    """Node-arc incidence of a directed 4-neighbour grid.

    Node (r, c) has index cols*r + c; every neighbour pair gets both arcs;
    arcs are sorted by (tail, head). Row v of A has +1 on arcs leaving v and
    -1 on arcs entering v. Returns (m, n, rowptr, colidx, val, tails, heads)."""
    tails, heads = [], []
    for r in range(rows):
        for c in range(cols):
            v = cols * r + c
            for dr, dc in ((-1, 0), (0, -1), (0, 1), (1, 0)):
                rr, cc = r + dr, c + dc
                if 0 <= rr < rows and 0 <= cc < cols:
                    tails.append(v)
                    heads.append(cols * rr + cc)
    tails = np.asarray(tails, dtype=np.int64)
    heads = np.asarray(heads, dtype=np.int64)
    order = np.lexsort((heads, tails))
    tails, heads = tails[order], heads[order]
    m, n = rows * cols, len(tails)
    ar = np.arange(n)
    rr = np.concatenate([tails, heads])
    cc = np.concatenate([ar, ar])
    vv = np.concatenate([np.ones(n), -np.ones(n)])
    order = np.lexsort((cc, rr))
    rr, cc, vv = rr[order], cc[order], vv[order]
    rowptr = np.zeros(m + 1, dtype=np.int32)
    np.cumsum(np.bincount(rr, minlength=m), out=rowptr[1:])
    return m, n, rowptr, cc.astype(np.int32), vv, tails, heads


def grid_mincost_batch(batch: int = 2048, rows: int = 32, cols: int = 32,
                       seed: int = 3000, costs: Optional[np.ndarray] = None) -> SharedBatch:
    """Min-cost-flow LPs sharing the grid incidence matrix.

    Per instance: arc costs U(1,10) (unless given, shape [batch, n]),
    capacities U(5,20), supply +k at a source and -k at a different sink,
    k ~ U{1..5}; rows are equalities A x = b, 0 <= x <= capacity."""
    m, n, rowptr, colidx, val, tails, heads = grid_incidence(rows, cols)
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 10.0, size=(batch, n)) if costs is None else np.asarray(costs, float)
    cap = rng.uniform(5.0, 20.0, size=(batch, n))
    src = rng.integers(0, m, size=batch)
    off = rng.integers(1, m, size=batch)
    snk = (src + off) % m
    k = rng.integers(1, 6, size=batch).astype(np.float64)
    b = np.zeros((batch, m))
    b[np.arange(batch), src] = k
    b[np.arange(batch), snk] = -k
    return SharedBatch(m, n, rowptr, colidx, val, c, b.copy(), b.copy(),
                       np.zeros((batch, n)), cap,
                       meta=dict(kind="grid_mincost", source=src, sink=snk, supply=k,
                                 tails=tails, heads=heads, grid=(rows, cols), seed=seed))


def shortest_path_learning(batch: int = 256, rows: int = 32, cols: int = 32, p: int = 5,
                           seed: int = 4000):
    """Learning-to-route workload: grid min-cost flows whose arc costs come
    from features. Per arc a of instance b: features f ~ N(0, I_p); the true
    cost is c_true = 1 + 9 sigmoid(w*' f) with w* ~ N(0, I_p) fixed by the
    seed (costs in [1, 10] as in the grid batch); the learner's initial
    weights W0 ~ N(0, 0.1^2). Capacities >= 5 >= supply never bind, so the
    optimum under c_true is supply x (shortest path).

    Returns (SharedBatch with c = c_true, features [batch, n, p], w_star, W0)."""
    rng = np.random.default_rng(seed)
    w_star = rng.normal(0.0, 1.0, size=p)
    W0 = rng.normal(0.0, 0.1, size=p)
    m, n, *_ = grid_incidence(rows, cols)
    feats = rng.normal(0.0, 1.0, size=(batch, n, p))
    c_true = 1.0 + 9.0 / (1.0 + np.exp(-(feats @ w_star)))
    sb = grid_mincost_batch(batch=batch, rows=rows, cols=cols, seed=seed + 1, costs=c_true)
    return sb, feats, w_star, W0


def ragged_planted_batch(batch: int = 1024, m_lo: int = 50, m_hi: int = 500,
                         density: float = 0.05, seed: int = 3500):
    """Planted sparse LPs of uneven size: m ~ U{m_lo..m_hi}, n = 2m."""
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo, m_hi + 1, size=batch)
    return [planted_sparse_lp(int(mi), 2 * int(mi), density=density,
                              seed=int(seed * 7919 + i)) for i, mi in enumerate(ms)]


def infeasible_lp(kind: str, m: int = 60, n: int = 120, seed: int = 0) -> LP:
    """LPs without an optimum, for the infeasibility tests.

    'duplicate_row': a planted sparse LP (x >= 0) plus a copy of one of its
        equality rows with the right-hand side moved by 1: no feasible point.
    'boxed_sum': m random dense equality rows satisfied by some x in [0, 1]^n,
        x boxed in [0, 1]^n, plus the row sum(x) = n + 1: no feasible point.
    'unbounded': a planted sparse LP plus a column u >= 0 with c_u = -1 whose
        entries are positive on some '>=' rows, negative on some '<=' rows and
        zero on the equality rows: feasible, and the objective decreases
        without bound along e_u, which moves A x into the interior of the
        one-sided rows."""
    rng = np.random.default_rng(seed)
    if kind == "boxed_sum":
        a = np.round(rng.standard_normal((m, n)), 3)
        x0 = rng.random(n)
        b = a @ x0
        a = np.vstack([a, np.ones((1, n))])
        b = np.append(b, n + 1.0)
        rowptr, colidx, val = csr_from_dense(a)
        c = np.round(rng.standard_normal(n), 3)
        return LP(m + 1, n, rowptr, colidx, val, c, b.copy(), b.copy(), np.zeros(n), np.ones(n),
                  meta=dict(kind="infeasible_boxed_sum", seed=seed))
    base = planted_sparse_lp(m, n, density=max(0.02, 4.0 / n), seed=seed)
    a = dense_from_csr(base.m, base.n, base.rowptr, base.colidx, base.val)
    if kind == "duplicate_row":
        eq = np.where(base.lc == base.uc)[0]
        i = int(eq[rng.integers(len(eq))])
        a = np.vstack([a, a[i:i + 1]])
        lc = np.append(base.lc, base.lc[i] + 1.0)
        uc = np.append(base.uc, base.uc[i] + 1.0)
        rowptr, colidx, val = csr_from_dense(a)
        return LP(m + 1, n, rowptr, colidx, val, base.c.copy(), lc, uc, base.lv.copy(), base.uv.copy(),
                  meta=dict(kind="infeasible_duplicate_row", seed=seed, row=i))
    if kind == "unbounded":
        ge = np.isfinite(base.lc) & ~np.isfinite(base.uc)
        le = ~np.isfinite(base.lc) & np.isfinite(base.uc)
        pick = rng.random(m) < 0.3
        mag = rng.uniform(0.5, 1.5, m)
        col = np.where(pick & ge, mag, 0.0) - np.where(pick & le, mag, 0.0)
        if not np.any(col):
            col[np.where(ge | le)[0][0]] = 1.0 if ge.any() else -1.0
        a = np.hstack([a, col[:, None]])
        rowptr, colidx, val = csr_from_dense(a)
        c = np.append(base.c, -1.0)
        return LP(m, n + 1, rowptr, colidx, val, c, base.lc.copy(), base.uc.copy(),
                  np.zeros(n + 1), np.full(n + 1, INF), meta=dict(kind="unbounded", seed=seed))
    raise ValueError(kind)


def contradict_row(lp: LP, seed: int = 0) -> LP:
    """A copy of a sparse LP plus a duplicate of one of its equality rows whose
    right-hand side is moved by 1: the same matrix shape and structure, no
    feasible point (works at any size; CSR append)."""
    rng = np.random.default_rng(seed)
    eq = np.where(np.isfinite(lp.lc) & (lp.lc == lp.uc) & (np.diff(lp.rowptr) > 0))[0]
    i = int(eq[rng.integers(len(eq))])
    a, b = int(lp.rowptr[i]), int(lp.rowptr[i + 1])
    rowptr = np.append(lp.rowptr, lp.rowptr[-1] + (b - a)).astype(np.int32)
    colidx = np.concatenate([lp.colidx, lp.colidx[a:b]]).astype(np.int32)
    val = np.concatenate([lp.val, lp.val[a:b]])
    return LP(lp.m + 1, lp.n, rowptr, colidx, val, lp.c, np.append(lp.lc, lp.lc[i] + 1.0),
              np.append(lp.uc, lp.uc[i] + 1.0), lp.lv, lp.uv,
              meta=dict(lp.meta, kind="contradicted_" + str(lp.meta.get("kind", "lp")), row=i))


def tiny_boxed_lp(m: int, n: int, seed: int) -> LP:
    """Tiny dense LP with finite boxes on every variable and mixed row types
    (=, <=, >=, two-sided), feasible by construction."""
    rng = np.random.default_rng(seed)
    a = np.round(rng.standard_normal((m, n)), 3)
    lv = -rng.uniform(0.0, 2.0, n)
    uv = rng.uniform(0.5, 2.0, n)
    x0 = lv + (uv - lv) * rng.random(n)
    ax = a @ x0
    kind = rng.integers(0, 4, size=m)
    lc = np.full(m, -INF)
    uc = np.full(m, INF)
    for i in range(m):
        if kind[i] == 0:
            lc[i] = uc[i] = ax[i]
        elif kind[i] == 1:
            uc[i] = ax[i] + rng.uniform(0, 1)
        elif kind[i] == 2:
            lc[i] = ax[i] - rng.uniform(0, 1)
        else:
            lc[i] = ax[i] - rng.uniform(0, 1)
            uc[i] = ax[i] + rng.uniform(0, 1)
    c = np.round(rng.standard_normal(n), 3)
    rowptr, colidx, val = csr_from_dense(a)
    return LP(m, n, rowptr, colidx, val, c, lc, uc, lv, uv,
              meta=dict(kind="tiny_boxed", seed=seed))


# ----------------------------------------------------------------------------
# QP


def portfolio_qp_batch(batch: int = 512, n: int = 500, rank: int = 20,
                       seed: int = 4500, shared_factor: bool = True):
    """Portfolio QPs: Q = F F' + diag(d), F ~ N(0, 0.1^2) [n, rank] (shared by
    the batch), d ~ U(0.01, 0.1), c ~ N(0, 0.05^2), sum(x) = 1, 0 <= x <= 0.1.

    Returns (F, d[B, n], c[B, n], A row pattern) as a dict."""
    rng = np.random.default_rng(seed)
    F = rng.normal(0.0, 0.1, size=(n, rank))
    d = rng.uniform(0.01, 0.1, size=(batch, n))
    c = rng.normal(0.0, 0.05, size=(batch, n))
    rowptr = np.array([0, n], dtype=np.int32)
    colidx = np.arange(n, dtype=np.int32)
    val = np.ones(n)
    return dict(F=F, d=d, c=c, m=1, n=n, rank=rank, rowptr=rowptr, colidx=colidx,
                val=val, lc=np.ones(1), uc=np.ones(1), lv=np.zeros(n),
                uv=np.full(n, 0.1), seed=seed)


def portfolio_instance(p: dict, b: int) -> LP:
    n = p["n"]
    return LP(1, n, p["rowptr"], p["colidx"], p["val"], p["c"][b].copy(),
              p["lc"].copy(), p["uc"].copy(), p["lv"].copy(), p["uv"].copy(),
              q_kind="lowrank", q_factor=p["F"], q_diag=p["d"][b].copy(),
              meta=dict(kind="portfolio", seed=p["seed"], index=b))


def infeasible_qp(kind: str, m: int = 40, n: int = 80, seed: int = 0) -> LP:
    """QPs without an optimum: the infeasible_lp family of the same kind with a
    convex Q = G G' (G ~ 0.3 N(0, 1), n x n/4, CSR) on its first n variables.
    The column added for 'unbounded' has no Q entries, so the objective is
    linear, and decreasing, along its ray."""
    lp = infeasible_lp(kind, m, n, seed)
    rng = np.random.default_rng(seed + 31)
    g = 0.3 * rng.standard_normal((n, max(1, n // 4)))
    q = np.zeros((lp.n, lp.n))
    q[:n, :n] = g @ g.T
    qr, qc, qv = csr_from_dense(q)
    lp.q_kind = "csr"
    lp.q_rowptr, lp.q_colidx, lp.q_val = qr, qc, qv
    lp.meta["kind"] = "qp_" + lp.meta.get("kind", kind)
    return lp


def mixed_qp_batch(kinds, m: int = 40, n: int = 80, rank: int = 4, seed: int = 0) -> SharedBatch:
    """A shared-A batch of QPs (Q_b = F F' + diag(d_b)) in which each instance
    is of the given kind: 'optimal', 'primal_infeasible' or 'dual_infeasible'.

    A is a planted sparse LP (x >= 0) plus a copy of one of its equality rows
    and a column u whose entries are positive on some '>=' rows, negative on
    some '<=' rows and zero elsewhere. F ~ 0.3 N(0, 1) has a zero row for u.
    'optimal': the copied row keeps its right-hand side, d ~ U(0.01, 0.1)
        everywhere (Q positive definite) and c_u = 1;
    'primal_infeasible': the same with the copy's right-hand side moved by 1;
    'dual_infeasible': consistent rows, d_u = 0 and c_u = -1, so the objective
        is linear and decreasing along e_u, a direction of the recession cone.
    The other costs are the planted ones plus 0.05 N(0, 1) per instance."""
    rng = np.random.default_rng(seed)
    base = planted_sparse_lp(m, n, density=max(0.02, 4.0 / n), seed=seed)
    a = dense_from_csr(base.m, base.n, base.rowptr, base.colidx, base.val)
    eq = np.where(base.lc == base.uc)[0]
    i = int(eq[rng.integers(len(eq))])
    ge = np.isfinite(base.lc) & ~np.isfinite(base.uc)
    le = ~np.isfinite(base.lc) & np.isfinite(base.uc)
    pick = rng.random(m) < 0.3
    mag = rng.uniform(0.5, 1.5, m)
    col = np.where(pick & ge, mag, 0.0) - np.where(pick & le, mag, 0.0)
    if not np.any(col):
        col[np.where(ge | le)[0][0]] = 1.0 if ge.any() else -1.0
    a = np.vstack([a, a[i:i + 1]])
    a = np.hstack([a, np.append(col, 0.0)[:, None]])
    rowptr, colidx, val = csr_from_dense(a)
    B, M, N = len(kinds), m + 1, n + 1
    F = np.zeros((N, rank))
    F[:n] = 0.3 * rng.standard_normal((n, rank))
    c = np.empty((B, N))
    lc = np.empty((B, M))
    uc = np.empty((B, M))
    d = np.empty((B, N))
    for b, kind in enumerate(kinds):
        if kind not in ("optimal", "primal_infeasible", "dual_infeasible"):
            raise ValueError(kind)
        shift = 1.0 if kind == "primal_infeasible" else 0.0
        lc[b] = np.append(base.lc, base.lc[i] + shift)
        uc[b] = np.append(base.uc, base.uc[i] + shift)
        c[b] = np.append(base.c + 0.05 * rng.standard_normal(n), -1.0 if kind == "dual_infeasible" else 1.0)
        d[b] = rng.uniform(0.01, 0.1, N)
        if kind == "dual_infeasible":
            d[b, n] = 0.0
    return SharedBatch(M, N, rowptr, colidx, val, c, lc, uc, np.zeros((B, N)), np.full((B, N), INF),
                       meta=dict(kind=np.array(list(kinds)), seed=seed, row=i), q_factor=F, q_diag=d)


def random_qp(m: int, n: int, seed: int, density: float = 0.3) -> LP:
    """Small random convex QP with boxes and mixed rows (CSR Q = G G' + eps I)."""
    lp = tiny_boxed_lp(m, n, seed)
    rng = np.random.default_rng(seed + 17)
    g = rng.standard_normal((n, max(1, n // 2)))
    g *= rng.random(g.shape) < max(density, 0.5)
    q = g @ g.T + 0.1 * np.eye(n)
    qr, qc, qv = csr_from_dense(q)
    lp.q_kind = "csr"
    lp.q_rowptr, lp.q_colidx, lp.q_val = qr, qc, qv
    lp.meta["kind"] = "random_qp"
    return lp
