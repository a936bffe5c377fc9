"""Helpers shared by the GPU parity tests."""

import numpy as np


def rel_inf(got, ref):
    """max |got - ref| / max(|ref|_inf, tiny): the per-vector parity metric."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def to_np(t):
    return t.detach().cpu().numpy()
