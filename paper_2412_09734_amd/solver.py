"""Thin Python binding over libpdhg's C ABI.

PyTorch provides device memory and the current stream; every step of the
method runs in the HIP kernels behind the ABI. There is no CPU fallback: if
the library is not built or no GPU is present, construction raises.
"""

from __future__ import annotations

import ctypes as C
from collections.abc import Sequence
from typing import Optional

import numpy as np
import torch

from . import _capi as capi


def _device(device=None) -> torch.device:
    if not torch.cuda.is_available():
        raise RuntimeError("libpdhg needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())


def _to_dev(a, dtype, dev) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device=dev, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(dev).contiguous()


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_ptr():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def options(**kw) -> capi.Options:
    o = capi.Options()
    capi.lib().pdhg_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Solver:
    """One LP (CSR constraint matrix) on the GPU.

    Arrays may be numpy arrays or torch tensors; they are copied to the
    device, handed to pdhg_create (which keeps its own scaled copy) and
    released."""

    def __init__(self, m, n, rowptr, colidx, val, c, lc, uc, lv, uv, *, q_format="none",
                 q_rowptr=None, q_colidx=None, q_val=None, q_dense=None, q_factor=None,
                 q_diag=None, a_dense=None, device=None, **opts):
        self.dev = _device(device)
        self.m, self.n = int(m), int(n)
        self._opts = options(**opts)
        self.qp = q_format != "none"
        with torch.cuda.device(self.dev):
            dense = a_dense is not None
            z32 = torch.zeros(1, dtype=torch.int32, device=self.dev)
            z64 = torch.zeros(1, dtype=torch.float64, device=self.dev)
            t = dict(rowptr=z32 if dense else _to_dev(rowptr, torch.int32, self.dev),
                     colidx=z32 if dense else _to_dev(colidx, torch.int32, self.dev),
                     val=z64 if dense else _to_dev(val, torch.float64, self.dev),
                     c=_to_dev(c, torch.float64, self.dev),
                     lc=_to_dev(lc, torch.float64, self.dev),
                     uc=_to_dev(uc, torch.float64, self.dev),
                     lv=_to_dev(lv, torch.float64, self.dev),
                     uv=_to_dev(uv, torch.float64, self.dev))
            p = capi.Problem()
            p.m, p.n = self.m, self.n
            p.a_format = capi.FMT_CSR
            p.a_rowptr, p.a_colidx, p.a_val = t["rowptr"].data_ptr(), t["colidx"].data_ptr(), t["val"].data_ptr()
            p.a_nnz = int(t["colidx"].numel())
            if dense:
                t["dense"] = _to_dev(a_dense, torch.float64, self.dev)
                p.a_format, p.a_dense, p.a_nnz = capi.FMT_DENSE, t["dense"].data_ptr(), 0
            p.c, p.lc, p.uc = t["c"].data_ptr(), t["lc"].data_ptr(), t["uc"].data_ptr()
            p.lv, p.uv = t["lv"].data_ptr(), t["uv"].data_ptr()
            p.q_format = capi.FMT_NONE
            if q_format == "csr":
                t["qr"], t["qc"], t["qv"] = (_to_dev(q_rowptr, torch.int32, self.dev),
                                             _to_dev(q_colidx, torch.int32, self.dev),
                                             _to_dev(q_val, torch.float64, self.dev))
                p.q_format, p.q_rowptr, p.q_colidx, p.q_val = (capi.FMT_CSR, t["qr"].data_ptr(),
                                                               t["qc"].data_ptr(), t["qv"].data_ptr())
                p.q_nnz = int(t["qc"].numel())
            elif q_format == "dense":
                t["qd"] = _to_dev(q_dense, torch.float64, self.dev)
                p.q_format, p.q_dense = capi.FMT_DENSE, t["qd"].data_ptr()
            elif q_format == "lowrank":
                t["qf"] = _to_dev(q_factor, torch.float64, self.dev)
                t["qg"] = _to_dev(q_diag, torch.float64, self.dev)
                p.q_format, p.q_factor, p.q_diag = (capi.FMT_LOWRANK_DIAG, t["qf"].data_ptr(),
                                                    t["qg"].data_ptr())
                p.q_rank = int(t["qf"].shape[1]) if t["qf"].dim() == 2 else 1
            elif q_format != "none":
                raise ValueError(f"unknown q_format {q_format}")
            p.mem = capi.MEM_DEVICE
            h = C.c_void_p()
            rc = capi.lib().pdhg_create(C.byref(p), C.byref(self._opts), _stream_ptr(), C.byref(h))
            capi.check(rc, "pdhg_create")
            self._h = h
        del t

    @classmethod
    def from_lp(cls, lp, **opts) -> "Solver":
        """From any object with m, n, rowptr, colidx, val, c, lc, uc, lv, uv
        (and optionally q_kind 'csr' / 'lowrank' with its Q arrays)."""
        q = {}
        kind = getattr(lp, "q_kind", "none")
        if kind == "csr":
            q = dict(q_format="csr", q_rowptr=lp.q_rowptr, q_colidx=lp.q_colidx, q_val=lp.q_val)
        elif kind == "lowrank":
            q = dict(q_format="lowrank", q_factor=lp.q_factor, q_diag=lp.q_diag)
        elif kind == "dense":
            q = dict(q_format="dense", q_dense=lp.q_dense)
        if getattr(lp, "dense", None) is not None:
            q["a_dense"] = lp.dense
        return cls(lp.m, lp.n, lp.rowptr, lp.colidx, lp.val, lp.c, lp.lc, lp.uc, lp.lv, lp.uv,
                   **q, **opts)

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().pdhg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _vec(self, v, length):
        if v is None:
            return None
        t = _to_dev(v, torch.float64, self.dev)
        if t.numel() != length:
            raise ValueError(f"expected a vector of length {length}, got {t.numel()}")
        return t

    def solve(self, x_init=None, y_init=None, out=None):
        """Solve; returns (x, y, info dict). out=(x, y) reuses device tensors."""
        xi, yi = self._vec(x_init, self.n), self._vec(y_init, self.m)
        if out is None:
            x = torch.empty(self.n, dtype=torch.float64, device=self.dev)
            y = torch.empty(max(self.m, 1), dtype=torch.float64, device=self.dev)
        else:
            x, y = out
        r = capi.Result()
        rc = capi.lib().pdhg_solve(self._h, _ptr(xi), _ptr(yi), _ptr(x), _ptr(y), C.byref(r))
        capi.check(rc, "pdhg_solve")
        return x, y[: self.m], r.as_dict()

    def debug_step(self, x, y, x0, y0, k, tau, sigma):
        """One iteration in the scaled space (original order)."""
        x, x0 = self._vec(x, self.n), self._vec(x0, self.n)
        y = self._vec(y, self.m) if self.m else torch.zeros(1, dtype=torch.float64, device=self.dev)
        y0 = self._vec(y0, self.m) if self.m else torch.zeros(1, dtype=torch.float64, device=self.dev)
        outs = [torch.empty(self.n, dtype=torch.float64, device=self.dev),
                torch.empty(max(self.m, 1), dtype=torch.float64, device=self.dev),
                torch.empty(self.n, dtype=torch.float64, device=self.dev),
                torch.empty(max(self.m, 1), dtype=torch.float64, device=self.dev)]
        rc = capi.lib().pdhg_debug_step(self._h, _ptr(x), _ptr(y), _ptr(x0), _ptr(y0), int(k),
                                        float(tau), float(sigma), *[_ptr(o) for o in outs])
        capi.check(rc, "pdhg_debug_step")
        return outs[0], outs[1][: self.m], outs[2], outs[3][: self.m]

    def debug_plain_step(self, x, y, x0, y0, k, tau, sigma):
        """One plain iteration (the solve's kernels between checks) in the
        scaled space (original order): the Halpern point (xnew, ynew)."""
        x, x0 = self._vec(x, self.n), self._vec(x0, self.n)
        y = self._vec(y, self.m) if self.m else torch.zeros(1, dtype=torch.float64, device=self.dev)
        y0 = self._vec(y0, self.m) if self.m else torch.zeros(1, dtype=torch.float64, device=self.dev)
        outs = [torch.empty(self.n, dtype=torch.float64, device=self.dev),
                torch.empty(max(self.m, 1), dtype=torch.float64, device=self.dev)]
        rc = capi.lib().pdhg_debug_plain_step(self._h, _ptr(x), _ptr(y), _ptr(x0), _ptr(y0), int(k),
                                              float(tau), float(sigma), *[_ptr(o) for o in outs])
        capi.check(rc, "pdhg_debug_plain_step")
        return outs[0], outs[1][: self.m]

    def debug_qp_step(self, x, y, xbar, ybar, k, omega):
        """One rAPDHG iteration in the scaled space (original order)."""
        z = lambda: torch.zeros(1, dtype=torch.float64, device=self.dev)  # noqa: E731
        x, xbar = self._vec(x, self.n), self._vec(xbar, self.n)
        y = self._vec(y, self.m) if self.m else z()
        ybar = self._vec(ybar, self.m) if self.m else z()
        outs = [torch.empty(self.n, dtype=torch.float64, device=self.dev),
                torch.empty(max(self.m, 1), dtype=torch.float64, device=self.dev),
                torch.empty(self.n, dtype=torch.float64, device=self.dev),
                torch.empty(max(self.m, 1), dtype=torch.float64, device=self.dev)]
        rc = capi.lib().pdhg_debug_qp_step(self._h, _ptr(x), _ptr(y), _ptr(xbar), _ptr(ybar),
                                           int(k), float(omega), *[_ptr(o) for o in outs])
        capi.check(rc, "pdhg_debug_qp_step")
        return outs[0], outs[1][: self.m], outs[2], outs[3][: self.m]

    def scaling(self) -> dict:
        dr = torch.empty(max(self.m, 1), dtype=torch.float64, device=self.dev)
        dc = torch.empty(self.n, dtype=torch.float64, device=self.dev)
        sc = (C.c_double * 4)()
        it = C.c_int32()
        rc = capi.lib().pdhg_get_scaling(self._h, _ptr(dr), _ptr(dc), sc, C.byref(it))
        capi.check(rc, "pdhg_get_scaling")
        return dict(dr=dr[: self.m], dc=dc, eta=sc[0], omega=sc[1], norm_a=sc[2], norm_q=sc[3],
                    power_iters=it.value)

    def update_data(self, c=None, lc=None, uc=None, lv=None, uv=None):
        t = [self._vec(c, self.n), self._vec(lc, self.m), self._vec(uc, self.m),
             self._vec(lv, self.n), self._vec(uv, self.n)]
        rc = capi.lib().pdhg_update_data(self._h, *[_ptr(a) for a in t])
        capi.check(rc, "pdhg_update_data")


class BatchResults(Sequence):
    """Per-instance results of a batch solve: the library's result array,
    each entry turned into a dict when it is read."""

    def __init__(self, arr):
        self._a = arr

    def __len__(self) -> int:
        return len(self._a)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self._a[k].as_dict() for k in range(*i.indices(len(self._a)))]
        i = int(i)
        if i < 0:
            i += len(self._a)
        if not 0 <= i < len(self._a):
            raise IndexError(i)
        return self._a[i].as_dict()

    def __add__(self, other):
        return list(self) + list(other)

    def __radd__(self, other):
        return list(other) + list(self)


class BatchSolver:
    """Many LPs solved in one persistent launch (pdhg_batch_*).

    Shared A: `c, lv, uv` are [B, n] and `lc, uc` [B, m]. Ragged: one
    block-diagonal CSR with `row_off`, `col_off` ([B+1]) and concatenated
    vectors (see `from_lps`). QPs (shared A only, rAPDHG): `q_factor` F [n, r]
    shared and `q_diag` d [B, n], Q_b = F F' + diag(d_b)."""

    def __init__(self, *, shared_a, batch, m, n, rowptr, colidx, val, c, lc, uc, lv, uv,
                 row_off=None, col_off=None, q_factor=None, q_diag=None, device=None,
                 threads=None, **opts):
        self.dev = _device(device)
        self.shared = bool(shared_a)
        self.batch, self.m, self.n = int(batch), int(m), int(n)
        self._opts = options(**opts)
        f64 = lambda a: _to_dev(a, torch.float64, self.dev).reshape(-1)  # noqa: E731
        i32 = lambda a: _to_dev(a, torch.int32, self.dev).reshape(-1)  # noqa: E731
        with torch.cuda.device(self.dev):
            t = dict(rowptr=i32(rowptr), colidx=i32(colidx), val=f64(val), c=f64(c), lc=f64(lc),
                     uc=f64(uc), lv=f64(lv), uv=f64(uv))
            if not self.shared:
                t["row_off"], t["col_off"] = i32(row_off), i32(col_off)
            p = capi.BatchProblem()
            p.batch, p.shared_a, p.m, p.n = self.batch, int(self.shared), self.m, self.n
            p.a_rowptr, p.a_colidx, p.a_val = (t["rowptr"].data_ptr(), t["colidx"].data_ptr(),
                                               t["val"].data_ptr())
            p.a_nnz = int(t["colidx"].numel())
            if not self.shared:
                p.row_off, p.col_off = t["row_off"].data_ptr(), t["col_off"].data_ptr()
            p.c, p.lc, p.uc = t["c"].data_ptr(), t["lc"].data_ptr(), t["uc"].data_ptr()
            p.lv, p.uv = t["lv"].data_ptr(), t["uv"].data_ptr()
            self.qp = q_factor is not None
            if self.qp:
                t["qf"] = _to_dev(q_factor, torch.float64, self.dev)
                t["qd"] = f64(q_diag)
                p.q_rank = int(t["qf"].shape[1]) if t["qf"].dim() == 2 else 1
                p.q_factor, p.q_diag = t["qf"].data_ptr(), t["qd"].data_ptr()
            p.mem = capi.MEM_DEVICE
            h = C.c_void_p()
            rc = capi.lib().pdhg_batch_create(C.byref(p), C.byref(self._opts), _stream_ptr(),
                                              C.byref(h))
            capi.check(rc, "pdhg_batch_create")
            self._h = h
            self.vec_n = int(t["c"].numel())
            self.vec_m = int(t["lc"].numel())
            if not self.shared:
                self.row_off = np.asarray(row_off, dtype=np.int64)
                self.col_off = np.asarray(col_off, dtype=np.int64)
        if threads is not None:
            self.set_launch(threads)

    @classmethod
    def from_shared(cls, sb, **opts) -> "BatchSolver":
        """From an object with m, n, rowptr, colidx, val and [B, .] vectors
        (and optionally q_factor [n, r] and q_diag [B, n])."""
        q = {}
        if getattr(sb, "q_factor", None) is not None:
            q = dict(q_factor=sb.q_factor, q_diag=sb.q_diag)
        return cls(shared_a=True, batch=sb.c.shape[0], m=sb.m, n=sb.n, rowptr=sb.rowptr,
                   colidx=sb.colidx, val=sb.val, c=sb.c, lc=sb.lc, uc=sb.uc, lv=sb.lv, uv=sb.uv,
                   **q, **opts)

    @classmethod
    def from_lps(cls, lps, **opts) -> "BatchSolver":
        """Ragged batch from a list of LP objects (block-diagonal concatenation)."""
        return cls(**cls.ragged_arrays(lps), **opts)

    @staticmethod
    def ragged_arrays(lps) -> dict:
        """Constructor arguments of the ragged batch of `lps` (host arrays)."""
        ms = np.array([lp.m for lp in lps], dtype=np.int64)
        ns = np.array([lp.n for lp in lps], dtype=np.int64)
        row_off = np.concatenate([[0], np.cumsum(ms)])
        col_off = np.concatenate([[0], np.cumsum(ns)])
        nnz_off = np.concatenate([[0], np.cumsum([int(lp.rowptr[-1]) for lp in lps])])
        rowptr = np.concatenate([lp.rowptr[:-1].astype(np.int64) + nnz_off[b] for b, lp in enumerate(lps)]
                                + [[nnz_off[-1]]])
        colidx = np.concatenate([lp.colidx.astype(np.int64) + col_off[b] for b, lp in enumerate(lps)])
        cat = lambda f: np.concatenate([getattr(lp, f) for lp in lps])  # noqa: E731
        return dict(shared_a=False, batch=len(lps), m=int(row_off[-1]), n=int(col_off[-1]),
                    rowptr=rowptr, colidx=colidx, val=cat("val"), c=cat("c"), lc=cat("lc"),
                    uc=cat("uc"), lv=cat("lv"), uv=cat("uv"), row_off=row_off, col_off=col_off)

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().pdhg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_launch(self, threads, workgroups=0):
        capi.check(capi.lib().pdhg_batch_set_launch(self._h, int(threads), int(workgroups)),
                   "pdhg_batch_set_launch")

    def autotune(self, iterations=256) -> int:
        best = C.c_int32()
        capi.check(capi.lib().pdhg_batch_autotune(self._h, int(iterations), C.byref(best)),
                   "pdhg_batch_autotune")
        return best.value

    def solve(self, x_init=None, y_init=None):
        """Returns (x, y, results): x [B, n] / y [B, m] for a shared A, flat
        concatenated vectors for a ragged batch; results is a sequence of
        dicts (BatchResults)."""
        xi = None if x_init is None else _to_dev(x_init, torch.float64, self.dev).reshape(-1)
        yi = None if y_init is None else _to_dev(y_init, torch.float64, self.dev).reshape(-1)
        x = torch.empty(self.vec_n, dtype=torch.float64, device=self.dev)
        y = torch.empty(max(self.vec_m, 1), dtype=torch.float64, device=self.dev)
        res = (capi.Result * self.batch)()
        rc = capi.lib().pdhg_batch_solve(self._h, _ptr(xi), _ptr(yi), _ptr(x), _ptr(y), res)
        capi.check(rc, "pdhg_batch_solve")
        out = BatchResults(res)
        y = y[: self.vec_m]
        if self.shared:
            return x.reshape(self.batch, self.n), y.reshape(self.batch, self.m), out
        return x, y, out

    def instance_slices(self, b):
        """(column slice, row slice) of instance b in the flat ragged vectors."""
        return (slice(int(self.col_off[b]), int(self.col_off[b + 1])),
                slice(int(self.row_off[b]), int(self.row_off[b + 1])))

    # -- differentiation by unrolling (LP batches) ---------------------------

    def update_data(self, c=None, lc=None, uc=None, lv=None, uv=None):
        """New per-instance vectors, laid out as at construction."""
        def dev(a, length):
            if a is None:
                return None
            t = _to_dev(a, torch.float64, self.dev).reshape(-1)
            if t.numel() != length:
                raise ValueError(f"expected {length} values, got {t.numel()}")
            return t
        t = [dev(c, self.vec_n), dev(lc, self.vec_m), dev(uc, self.vec_m),
             dev(lv, self.vec_n), dev(uv, self.vec_n)]
        rc = capi.lib().pdhg_batch_update_data(self._h, *[_ptr(a) for a in t])
        capi.check(rc, "pdhg_batch_update_data")

    def unrolled(self, T, replay=False):
        """Exactly T iterations per instance; returns the PDHG point of the
        last one for LPs, the averages (xbar, ybar) for QPs (shaped like
        solve()). replay=True reuses the schedule of the last replay=False
        call."""
        x = torch.empty(self.vec_n, dtype=torch.float64, device=self.dev)
        y = torch.empty(max(self.vec_m, 1), dtype=torch.float64, device=self.dev)
        rc = capi.lib().pdhg_batch_unrolled_forward(self._h, int(T), int(bool(replay)), _ptr(x), _ptr(y))
        capi.check(rc, "pdhg_batch_unrolled_forward")
        y = y[: self.vec_m]
        if self.shared:
            return x.reshape(self.batch, self.n), y.reshape(self.batch, self.m)
        return x, y

    def backward(self, gx, gy=None):
        """Gradients (gc, glc, guc) of <gx, x_T> + <gy, y_T> for the last
        unrolled call; QP batches return (gc, glc, guc, gd)."""
        gxt = _to_dev(gx, torch.float64, self.dev).reshape(-1)
        gyt = None if gy is None else _to_dev(gy, torch.float64, self.dev).reshape(-1)
        gc = torch.empty(self.vec_n, dtype=torch.float64, device=self.dev)
        glc = torch.empty(max(self.vec_m, 1), dtype=torch.float64, device=self.dev)
        guc = torch.empty(max(self.vec_m, 1), dtype=torch.float64, device=self.dev)
        gd = torch.empty(self.vec_n, dtype=torch.float64, device=self.dev) if self.qp else None
        rc = capi.lib().pdhg_batch_unrolled_backward(self._h, _ptr(gxt), _ptr(gyt), _ptr(gc),
                                                     _ptr(glc), _ptr(guc), _ptr(gd))
        capi.check(rc, "pdhg_batch_unrolled_backward")
        glc, guc = glc[: self.vec_m], guc[: self.vec_m]
        if self.shared:
            out = (gc.reshape(self.batch, self.n), glc.reshape(self.batch, self.m),
                   guc.reshape(self.batch, self.m))
            if self.qp:
                out = out + (gd.reshape(self.batch, self.n),)
            return out
        return gc, glc, guc


class UnrolledLP(torch.autograd.Function):
    """x_T(c): T unrolled r2HPDHG iterations of a batch, differentiable in c.

    forward(c, solver, T) sets the batch objective to c, runs the unrolled
    iterations (recording the schedule) and returns x_T; backward runs the
    hand-written adjoint kernel."""

    @staticmethod
    def forward(ctx, c, solver, T):
        solver.update_data(c=c.detach())
        x, _ = solver.unrolled(T)
        ctx.solver = solver
        ctx.shape = c.shape
        return x.reshape(c.shape)

    @staticmethod
    def backward(ctx, gx):
        gc = ctx.solver.backward(gx.detach().contiguous())[0]
        return gc.reshape(ctx.shape), None, None
