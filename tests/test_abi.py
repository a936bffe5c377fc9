"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/pdhg.h declares, and rejects bad arguments before
touching the device."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdhg_[a-z_0-9]+)\s*\(", text)))


def _lib():
    from paper_2412_09734_amd._build import LIB, build
    if not os.path.exists(LIB):
        build()
    return C.CDLL(LIB)


def test_library_exports_every_declared_symbol():
    names = _declared("pdhg.h")
    assert "pdhg_create" in names and "pdhg_solve" in names
    lib = _lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2412_09734_amd import _capi
    assert set(_declared("pdhg.h")) == set(_capi.SIGNATURES)


def test_struct_layouts_match_header():
    """Field order and count of the ctypes mirrors equal the C structs."""
    from paper_2412_09734_amd import _capi
    text = open(os.path.join(ROOT, "include", "pdhg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    for cname, py in (("pdhg_problem", _capi.Problem), ("pdhg_options", _capi.Options),
                      ("pdhg_result", _capi.Result)):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", text).group(1)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            decl = re.sub(r"\b(const|int32_t|int64_t|double)\b", "", decl).replace("*", "")
            fields += [f.strip() for f in decl.split(",") if f.strip()]
        assert fields == [f for f, _ in py._fields_], cname


def test_defaults_and_argument_errors_without_gpu():
    from paper_2412_09734_amd import _capi
    lib = _capi.lib()
    o = _capi.Options()
    lib.pdhg_options_default(C.byref(o))
    assert o.eps == 1e-4 and o.check_every == 64 and o.ruiz_iters == 10
    assert o.display_frequency == 10 and o.iteration_limit == 2**63 - 1
    assert lib.pdhg_version() >= 100
    h = C.c_void_p()
    assert lib.pdhg_create(None, None, None, C.byref(h)) == -1
    assert b"NULL" in lib.pdhg_last_error()
    p = _capi.Problem()
    p.m, p.n = -1, 3
    assert lib.pdhg_create(C.byref(p), None, None, C.byref(h)) == -1
    p.m, p.n = 2, 3
    p.a_format = _capi.FMT_CSR
    p.mem = 7
    assert lib.pdhg_create(C.byref(p), None, None, C.byref(h)) == -1
    assert lib.pdhg_solve(None, None, None, None, None, None) == -1
    lib.pdhg_destroy(None)


def test_build_entry_compiles(tmp_path):
    """__graft_entry__.build() compiles the HIP library and the oracle."""
    import importlib
    import __graft_entry__ as g
    importlib.reload(g)
    g.build()
    from paper_2412_09734_amd._build import LIB
    assert os.path.exists(LIB)
