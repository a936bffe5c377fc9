"""Loss heads of the end-to-end learning pipelines, bound to libpdhg's
pdhg_linear_costs / pdhg_regret / pdhg_linear_costs_backward / pdhg_qp_value
and the LP surrogates pdhg_spo_plus_costs / pdhg_spo_plus / pdhg_pfy_costs /
pdhg_pfy.
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


def linear_costs_backward_noalloc(f, gc, gW, device=None) -> torch.Tensor:
    """linear_costs_backward into a caller-provided gW [p], with no device
    allocation (static partial-sum array; p <= 64); returns gW."""
    dev = _device(device)
    ft, gt = _f64(f, dev), _f64(gc, dev)
    B, n, p = ft.shape
    capi.check(capi.lib().pdhg_linear_costs_backward_noalloc(B, n, p, _ptr(ft), _ptr(gt), _ptr(gW),
                                                             _stream_ptr()),
               "pdhg_linear_costs_backward_noalloc")
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


def spo_plus_costs(c_hat, c_true, device=None) -> torch.Tensor:
    """Costs of the SPO+ inner problem, 2 c_hat - c_true [B, n]."""
    dev = _device(device)
    ch, ct = _f64(c_hat, dev), _f64(c_true, dev)
    B, n = ch.shape
    out = torch.empty(B, n, dtype=torch.float64, device=dev)
    capi.check(capi.lib().pdhg_spo_plus_costs(B, n, _ptr(ch), _ptr(ct), _ptr(out), _stream_ptr()),
               "pdhg_spo_plus_costs")
    return out


def spo_plus(c_hat, c_true, w_star, z_star, w_tilde, device=None):
    """(loss [B], subgradient [B, n]) of SPO+; w_star optimal under c_true with
    value z_star, w_tilde optimal under 2 c_hat - c_true."""
    dev = _device(device)
    ch, ct, ws, wt = (_f64(a, dev) for a in (c_hat, c_true, w_star, w_tilde))
    zs = _f64(z_star, dev).reshape(-1)
    B, n = ch.shape
    loss = torch.empty(B, dtype=torch.float64, device=dev)
    grad = torch.empty(B, n, dtype=torch.float64, device=dev)
    capi.check(capi.lib().pdhg_spo_plus(B, n, _ptr(ch), _ptr(ct), _ptr(ws), _ptr(zs), _ptr(wt), _ptr(loss),
                                        _ptr(grad), _stream_ptr()), "pdhg_spo_plus")
    return loss, grad


def pfy_costs(c_hat, Z, eps, device=None) -> torch.Tensor:
    """Perturbed costs [B, M, n]: c_hat[b] + eps Z[b, m]."""
    dev = _device(device)
    ch, Zt = _f64(c_hat, dev), _f64(Z, dev)
    B, M, n = Zt.shape
    out = torch.empty(B, M, n, dtype=torch.float64, device=dev)
    capi.check(capi.lib().pdhg_pfy_costs(B, M, n, _ptr(ch), _ptr(Zt), float(eps), _ptr(out), _stream_ptr()),
               "pdhg_pfy_costs")
    return out


def pfy(c_hat, w_star, Z, eps, w_samples, device=None):
    """(loss up to a constant [B], gradient [B, n]) of the perturbed
    Fenchel-Young loss from samples w_samples [B, M, n] optimal under
    pfy_costs(c_hat, Z, eps)."""
    dev = _device(device)
    ch, ws, Zt, wm = (_f64(a, dev) for a in (c_hat, w_star, Z, w_samples))
    B, M, n = Zt.shape
    loss = torch.empty(B, dtype=torch.float64, device=dev)
    grad = torch.empty(B, n, dtype=torch.float64, device=dev)
    capi.check(capi.lib().pdhg_pfy(B, M, n, _ptr(ch), _ptr(ws), _ptr(Zt), float(eps), _ptr(wm), _ptr(loss),
                                   _ptr(grad), _stream_ptr()), "pdhg_pfy")
    return loss, grad
