"""Python access to the plain C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke test and the
benchmark's CPU-baseline leg use this module; the GPU library never does.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "unsolved", 1: "optimal", 2: "primal_infeasible", 3: "dual_infeasible", 4: "iteration_limit",
          6: "numerical_error"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FMA contraction, OpenMP
    for the products)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
               "-Wall", "-Wno-unused-function", os.path.join(_HERE, "oracle.c"),
               "-o", _SO + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class Problem(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32),
                ("rowptr", C.c_void_p), ("colidx", C.c_void_p), ("val", C.c_void_p),
                ("dense", C.c_void_p),
                ("c", C.c_void_p), ("lc", C.c_void_p), ("uc", C.c_void_p),
                ("lv", C.c_void_p), ("uv", C.c_void_p),
                ("q_kind", C.c_int32),
                ("q_rowptr", C.c_void_p), ("q_colidx", C.c_void_p), ("q_val", C.c_void_p),
                ("q_rank", C.c_int32), ("q_factor", C.c_void_p), ("q_diag", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("eps", C.c_double), ("iteration_limit", C.c_int64),
                ("check_every", C.c_int32), ("ruiz_iters", C.c_int32),
                ("pock_chambolle", C.c_int32), ("gamma", C.c_double),
                ("step_safety", C.c_double), ("restart_sufficient", C.c_double),
                ("restart_necessary", C.c_double), ("restart_artificial", C.c_double),
                ("power_tol", C.c_double), ("power_max_iters", C.c_int32),
                ("verbose", C.c_int32), ("eps_primal_infeasible", C.c_double),
                ("eps_dual_infeasible", C.c_double), ("feasibility_polishing", C.c_int32),
                ("eps_feas_polish", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int64), ("restarts", C.c_int64),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double),
                ("rel_primal", C.c_double), ("rel_dual", C.c_double),
                ("rel_gap", C.c_double), ("kkt", C.c_double),
                ("abs_primal", C.c_double), ("abs_dual", C.c_double), ("abs_gap", C.c_double),
                ("eta", C.c_double), ("omega", C.c_double), ("norm_a", C.c_double),
                ("norm_q", C.c_double), ("power_iters", C.c_int32),
                ("polish_iterations", C.c_int64)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        P = C.c_void_p
        L.orc_default_options.argtypes = [C.POINTER(Options)]
        L.orc_create.argtypes = [C.POINTER(Problem), C.POINTER(Options)]
        L.orc_create.restype = P
        L.orc_destroy.argtypes = [P]
        L.orc_scaling.argtypes = [P, P, P, P, P, P, P, P]
        L.orc_scaled_vectors.argtypes = [P] * 6
        L.orc_lp_step.argtypes = [P, P, P, P, P, C.c_int64, C.c_double, C.c_double,
                                  C.c_double, P, P, P, P]
        L.orc_qp_step.argtypes = [P, P, P, P, P, C.c_int64, C.c_double, P, P, P, P]
        L.orc_fixed_point_residual.argtypes = [P, P, P, P, P, C.c_double, C.c_double]
        L.orc_fixed_point_residual.restype = C.c_double
        L.orc_kkt.argtypes = [C.POINTER(Problem), P, P, C.POINTER(Result)]
        L.orc_solve.argtypes = [P, P, P, P, P, C.POINTER(Result)]
        L.orc_solve.restype = C.c_int
        L.orc_unrolled_lp.argtypes = [P, C.c_int64, P, P, P, P, P, P]
        L.orc_unrolled_lp.restype = C.c_int
        L.orc_unrolled_lp_backward.argtypes = [P, C.c_int64, P, P, P, P, P, P, P]
        L.orc_unrolled_lp_backward.restype = C.c_int
        L.orc_pin_steps.argtypes = [P, C.c_double, C.c_double]
        L.orc_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads(1)   # one thread unless a caller asks for more (set_threads)
        L.orc_unrolled_qp.argtypes = [P, C.c_int64, P, P, P, P, P, P]
        L.orc_unrolled_qp.restype = C.c_int
        L.orc_unrolled_qp_backward.argtypes = [P, C.c_int64, P, P, P, P, P, P, P, P]
        L.orc_unrolled_qp_backward.restype = C.c_int
        _lib = L
    return _lib


def default_options(**kw) -> Options:
    o = Options()
    lib().orc_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


@dataclass
class _Keep:
    arrays: list


def make_problem(lp):
    """Build the C problem struct for a gen.LP (keeps the arrays alive)."""
    keep = []

    def k(a):
        keep.append(a)
        return _ptr(a)

    p = Problem()
    p.m, p.n = lp.m, lp.n
    if lp.dense is not None:
        p.dense = k(_f64(lp.dense))
    else:
        p.rowptr = k(_i32(lp.rowptr))
        p.colidx = k(_i32(lp.colidx))
        p.val = k(_f64(lp.val))
    p.c, p.lc, p.uc = k(_f64(lp.c)), k(_f64(lp.lc)), k(_f64(lp.uc))
    p.lv, p.uv = k(_f64(lp.lv)), k(_f64(lp.uv))
    if lp.q_kind == "csr":
        p.q_kind = 1
        p.q_rowptr, p.q_colidx, p.q_val = k(_i32(lp.q_rowptr)), k(_i32(lp.q_colidx)), k(_f64(lp.q_val))
    elif lp.q_kind == "lowrank":
        p.q_kind = 2
        f = _f64(lp.q_factor)
        p.q_rank = f.shape[1]
        p.q_factor = k(f)
        p.q_diag = k(_f64(lp.q_diag))
    return p, _Keep(keep)


def kkt(lp, x, y) -> dict:
    p, keep = make_problem(lp)
    x = _f64(x)
    y = _f64(y) if lp.m else np.zeros(1)
    r = Result()
    lib().orc_kkt(C.byref(p), _ptr(x), _ptr(y), C.byref(r))
    del keep
    return r.as_dict()


class Oracle:
    """Scaled problem + solver state owned by the C oracle."""

    def __init__(self, lp, **opts):
        self.lp = lp
        self.opts = default_options(**opts)
        self._p, self._keep = make_problem(lp)
        self._ctx = lib().orc_create(C.byref(self._p), C.byref(self.opts))
        if not self._ctx:
            raise ValueError("oracle rejected the problem (invalid input)")
        self.m, self.n = lp.m, lp.n

    def close(self):
        if self._ctx:
            lib().orc_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def scaling(self) -> dict:
        dr = np.zeros(max(self.m, 1))
        dc = np.zeros(self.n)
        vals = [C.c_double() for _ in range(4)]
        it = C.c_int32()
        lib().orc_scaling(self._ctx, _ptr(dr), _ptr(dc), *[C.byref(v) for v in vals], C.byref(it))
        return dict(dr=dr[: self.m], dc=dc, eta=vals[0].value, omega=vals[1].value,
                    norm_a=vals[2].value, norm_q=vals[3].value, power_iters=it.value)

    def pin_steps(self, eta, norm_q):
        lib().orc_pin_steps(self._ctx, float(eta), float(norm_q))

    def scaled_vectors(self) -> dict:
        out = dict(c=np.zeros(self.n), lc=np.zeros(max(self.m, 1)), uc=np.zeros(max(self.m, 1)),
                   lv=np.zeros(self.n), uv=np.zeros(self.n))
        lib().orc_scaled_vectors(self._ctx, *[_ptr(out[k]) for k in ("c", "lc", "uc", "lv", "uv")])
        out["lc"] = out["lc"][: self.m]
        out["uc"] = out["uc"][: self.m]
        return out

    def lp_step(self, x, y, x0, y0, k, tau, sigma, gamma=1.0):
        x, y, x0, y0 = map(_f64, (x, y, x0, y0))
        mm = max(self.m, 1)
        xh, xn = np.zeros(self.n), np.zeros(self.n)
        yh, yn = np.zeros(mm), np.zeros(mm)
        if self.m == 0:
            y = y0 = np.zeros(1)
        lib().orc_lp_step(self._ctx, _ptr(x), _ptr(y), _ptr(x0), _ptr(y0), int(k), float(tau),
                          float(sigma), float(gamma), _ptr(xh), _ptr(yh), _ptr(xn), _ptr(yn))
        return xh, yh[: self.m], xn, yn[: self.m]

    def qp_step(self, x, y, xbar, ybar, k, omega):
        x, y, xbar, ybar = map(_f64, (x, y, xbar, ybar))
        outs = [np.zeros(self.n), np.zeros(max(self.m, 1)), np.zeros(self.n), np.zeros(max(self.m, 1))]
        lib().orc_qp_step(self._ctx, _ptr(x), _ptr(y), _ptr(xbar), _ptr(ybar), int(k),
                          float(omega), *[_ptr(a) for a in outs])
        return outs[0], outs[1][: self.m], outs[2], outs[3][: self.m]

    def fixed_point_residual(self, x, y, xh, yh, tau, sigma) -> float:
        x, y, xh, yh = map(_f64, (x, y, xh, yh))
        return lib().orc_fixed_point_residual(self._ctx, _ptr(x), _ptr(y), _ptr(xh), _ptr(yh),
                                               float(tau), float(sigma))

    def solve(self, x_init=None, y_init=None):
        x = np.zeros(self.n)
        y = np.zeros(max(self.m, 1))
        r = Result()
        xi, yi = _f64(x_init), _f64(y_init)
        lib().orc_solve(self._ctx, _ptr(xi), _ptr(yi), _ptr(x), _ptr(y), C.byref(r))
        return x, y[: self.m], r.as_dict()

    def unrolled(self, T, sched_restart=None, sched_omega=None):
        x = np.zeros(self.n)
        y = np.zeros(max(self.m, 1))
        rec_r = np.zeros(T, dtype=np.uint8)
        rec_w = np.zeros(T)
        sr = None if sched_restart is None else np.ascontiguousarray(sched_restart, dtype=np.uint8)
        sw = _f64(sched_omega)
        rc = lib().orc_unrolled_lp(self._ctx, int(T), _ptr(sr), _ptr(sw), _ptr(rec_r), _ptr(rec_w),
                                   _ptr(x), _ptr(y))
        if rc != 0:
            raise ValueError("unrolled forward rejected")
        return x, y[: self.m], rec_r, rec_w

    def unrolled_qp(self, T, sched_restart=None, sched_omega=None):
        x = np.zeros(self.n)
        y = np.zeros(max(self.m, 1))
        rec_r = np.zeros(T, dtype=np.uint8)
        rec_w = np.zeros(T)
        sr = None if sched_restart is None else np.ascontiguousarray(sched_restart, dtype=np.uint8)
        sw = _f64(sched_omega)
        rc = lib().orc_unrolled_qp(self._ctx, int(T), _ptr(sr), _ptr(sw), _ptr(rec_r), _ptr(rec_w),
                                   _ptr(x), _ptr(y))
        if rc != 0:
            raise ValueError("unrolled QP forward rejected")
        return x, y[: self.m], rec_r, rec_w

    def backward_qp(self, T, sched_restart, sched_omega, gx, gy):
        sr = np.ascontiguousarray(sched_restart, dtype=np.uint8)
        sw = _f64(sched_omega)
        gx = _f64(gx)
        gy = _f64(gy) if self.m else np.zeros(1)
        gc, gd = np.zeros(self.n), np.zeros(self.n)
        glc = np.zeros(max(self.m, 1))
        guc = np.zeros(max(self.m, 1))
        rc = lib().orc_unrolled_qp_backward(self._ctx, int(T), _ptr(sr), _ptr(sw), _ptr(gx),
                                            _ptr(gy), _ptr(gc), _ptr(glc), _ptr(guc), _ptr(gd))
        if rc != 0:
            raise ValueError("unrolled QP backward rejected")
        return gc, glc[: self.m], guc[: self.m], gd

    def backward(self, T, sched_restart, sched_omega, gx, gy):
        sr = np.ascontiguousarray(sched_restart, dtype=np.uint8)
        sw = _f64(sched_omega)
        gx = _f64(gx)
        gy = _f64(gy) if self.m else np.zeros(1)
        gc = np.zeros(self.n)
        glc = np.zeros(max(self.m, 1))
        guc = np.zeros(max(self.m, 1))
        rc = lib().orc_unrolled_lp_backward(self._ctx, int(T), _ptr(sr), _ptr(sw), _ptr(gx),
                                            _ptr(gy), _ptr(gc), _ptr(glc), _ptr(guc))
        if rc != 0:
            raise ValueError("unrolled backward rejected")
        return gc, glc[: self.m], guc[: self.m]


def threads() -> int:
    """Threads the oracle's products use (OpenMP; 0 when built without it)."""
    return int(lib().orc_threads())


def set_threads(t: int) -> None:
    """Run the oracle's products on t threads (results do not depend on t)."""
    lib().orc_set_threads(int(t))
