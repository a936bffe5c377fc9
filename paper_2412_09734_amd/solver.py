"""Thin Python binding over libpdhg's C ABI.

PyTorch provides device memory and the current stream; every step of the
method runs in the HIP kernels behind the ABI. There is no CPU fallback: if
the library is not built or no GPU is present, construction raises.
"""

from __future__ import annotations

import ctypes as C
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

    def __init__(self, m, n, rowptr, colidx, val, c, lc, uc, lv, uv, *, device=None, **opts):
        self.dev = _device(device)
        self.m, self.n = int(m), int(n)
        self._opts = options(**opts)
        with torch.cuda.device(self.dev):
            t = dict(rowptr=_to_dev(rowptr, torch.int32, self.dev),
                     colidx=_to_dev(colidx, torch.int32, self.dev),
                     val=_to_dev(val, torch.float64, self.dev),
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
            p.c, p.lc, p.uc = t["c"].data_ptr(), t["lc"].data_ptr(), t["uc"].data_ptr()
            p.lv, p.uv = t["lv"].data_ptr(), t["uv"].data_ptr()
            p.q_format = capi.FMT_NONE
            p.mem = capi.MEM_DEVICE
            h = C.c_void_p()
            rc = capi.lib().pdhg_create(C.byref(p), C.byref(self._opts), _stream_ptr(), C.byref(h))
            capi.check(rc, "pdhg_create")
            self._h = h
        del t

    @classmethod
    def from_lp(cls, lp, **opts) -> "Solver":
        """From any object with m, n, rowptr, colidx, val, c, lc, uc, lv, uv."""
        return cls(lp.m, lp.n, lp.rowptr, lp.colidx, lp.val, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, **opts)

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
