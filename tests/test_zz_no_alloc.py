"""The allocation-free weight gradient (pdhg_linear_costs_backward_noalloc)
against pdhg_linear_costs_backward, through the C ABI. Both run the same two
kernels over the same partial-sum layout, so the outputs must be equal bit for
bit: on consecutive calls (the second one smaller, so the static array still
holds the first call's partials), on the caller's stream and on the NULL
stream. Feature counts beyond the static array are rejected."""

import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_09734_amd import _capi as capi
    return capi.lib()


def _call(lib, name, f, gc, gW, stream):
    B, n, p = f.shape
    return getattr(lib, name)(B, n, p, C.c_void_p(f.data_ptr()), C.c_void_p(gc.data_ptr()),
                              C.c_void_p(gW.data_ptr()), C.c_void_p(stream) if stream else None)


def test_noalloc_matches_allocating_entry_point(lib):
    import torch
    cases = [(256, 3968, 5, 0, "caller"), (3, 17, 2, 1, "caller"), (64, 500, 64, 2, "null"),
             (1, 1, 1, 3, "caller")]
    for B, n, p, seed, which in cases:
        print(f"case: weight gradient B={B} n={n} p={p} stream={which}", file=sys.stderr, flush=True)
        rng = np.random.default_rng(seed)
        fh, gh = rng.standard_normal((B, n, p)), rng.standard_normal((B, n))
        f = torch.tensor(fh, dtype=torch.float64, device="cuda")
        gc = torch.tensor(gh, dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream if which == "caller" else 0
        ref = torch.full((p,), float("nan"), dtype=torch.float64, device="cuda")
        got = torch.full((p,), float("nan"), dtype=torch.float64, device="cuda")
        assert _call(lib, "pdhg_linear_costs_backward", f, gc, ref, stream) == 0
        assert _call(lib, "pdhg_linear_costs_backward_noalloc", f, gc, got, stream) == 0
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        np.testing.assert_array_equal(g, r)
        exact = np.einsum("bn,bnp->p", gh, fh)
        scale = np.einsum("bn,bnp->p", np.abs(gh), np.abs(fh))
        assert np.all(np.abs(g - exact) <= 1e-13 * scale + 1e-300), (g, exact)


def test_noalloc_rejects_too_many_features(lib):
    import torch
    f = torch.zeros((2, 3, 65), dtype=torch.float64, device="cuda")
    gc = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    gW = torch.zeros(65, dtype=torch.float64, device="cuda")
    rc = _call(lib, "pdhg_linear_costs_backward_noalloc", f, gc, gW, 0)
    assert rc == -1
    assert b"64" in lib.pdhg_last_error()
