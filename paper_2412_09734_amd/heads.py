"""Loss heads of the end-to-end learning pipelines, bound to libpdhg's
pdhg_linear_costs / pdhg_regret / pdhg_linear_costs_backward / pdhg_qp_value.
Argument marshalling only; the arithmetic runs in the HIP kernels."""

from __future__ import annotations

import torch

from . import _capi as capi
from .solver import _device, _ptr, _stream_ptr, _to_dev


def _f64(a, dev):
    return _to_dev(a, torch.float64, dev)


def linear_costs(f, W, device=None) -> torch.Tensor:
    """c_hat [B, n] = f [B, n, p] @ W [p]."""
    dev = _device(device)
    ft, Wt = _f64(f, dev), _f64(W, dev).reshape(-1)
    B, n, p = ft.shape
    c = torch.empty(B, n, dtype=torch.float64, device=dev)
    capi.check(capi.lib().pdhg_linear_costs(B, n, p, _ptr(ft), _ptr(Wt), _ptr(c), _stream_ptr()),
               "pdhg_linear_costs")
    return c


def regret(c_true, x, v_star, device=None) -> torch.Tensor:
    """loss [B] = sum_a c_true[b, a] x[b, a] - v_star[b]."""
    dev = _device(device)
    ct, xt, vs = _f64(c_true, dev), _f64(x, dev), _f64(v_star, dev).reshape(-1)
    B, n = ct.shape
    loss = torch.empty(B, dtype=torch.float64, device=dev)
    capi.check(capi.lib().pdhg_regret(B, n, _ptr(ct), _ptr(xt), _ptr(vs), _ptr(loss), _stream_ptr()),
               "pdhg_regret")
    return loss


def linear_costs_backward(f, gc, device=None) -> torch.Tensor:
    """gW [p] = sum_{b, a} gc[b, a] f[b, a, :]."""
    dev = _device(device)
    ft, gt = _f64(f, dev), _f64(gc, dev)
    B, n, p = ft.shape
    gW = torch.empty(p, dtype=torch.float64, device=dev)
    capi.check(capi.lib().pdhg_linear_costs_backward(B, n, p, _ptr(ft), _ptr(gt), _ptr(gW),
                                                     _stream_ptr()), "pdhg_linear_costs_backward")
    return gW


def qp_value(F, d, c, x, grad=True, device=None):
    """(value [B], gradient [B, n] or None) of 1/2 x'(F F' + diag d)x + c'x."""
    dev = _device(device)
    Ft, dt, ct, xt = _f64(F, dev), _f64(d, dev), _f64(c, dev), _f64(x, dev)
    B, n = ct.shape
    r = int(Ft.shape[1]) if Ft.dim() == 2 else 0
    value = torch.empty(B, dtype=torch.float64, device=dev)
    gx = torch.empty(B, n, dtype=torch.float64, device=dev) if grad else None
    capi.check(capi.lib().pdhg_qp_value(B, n, r, _ptr(Ft), _ptr(dt), _ptr(ct), _ptr(xt), _ptr(value),
                                        _ptr(gx), _stream_ptr()), "pdhg_qp_value")
    return value, gx
