"""ctypes mirror of include/pdhg.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

from ._build import LIB

PDHG_OK = 0
ERRORS = {0: "ok", -1: "invalid argument", -2: "invalid input", -3: "out of memory",
          -4: "HIP error", -5: "unsupported"}
STATUS = {0: "unsolved", 1: "optimal", 2: "primal_infeasible", 3: "dual_infeasible",
          4: "iteration_limit", 5: "time_limit", 6: "numerical_error"}
FMT_NONE, FMT_CSR, FMT_DENSE, FMT_LOWRANK_DIAG = 0, 1, 2, 3
MEM_HOST, MEM_DEVICE = 0, 1

P = C.c_void_p


class Problem(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("a_format", C.c_int32),
                ("a_rowptr", P), ("a_colidx", P), ("a_val", P), ("a_nnz", C.c_int64),
                ("a_dense", P),
                ("c", P), ("lc", P), ("uc", P), ("lv", P), ("uv", P),
                ("q_format", C.c_int32), ("q_rowptr", P), ("q_colidx", P), ("q_val", P),
                ("q_nnz", C.c_int64), ("q_dense", P), ("q_rank", C.c_int32),
                ("q_factor", P), ("q_diag", P), ("mem", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("eps", C.c_double), ("iteration_limit", C.c_int64),
                ("time_limit_s", C.c_double), ("check_every", C.c_int32),
                ("ruiz_iters", C.c_int32), ("pock_chambolle", C.c_int32),
                ("gamma", C.c_double), ("step_safety", C.c_double),
                ("restart_sufficient", C.c_double), ("restart_necessary", C.c_double),
                ("restart_artificial", C.c_double), ("power_tol", C.c_double),
                ("power_max_iters", C.c_int32), ("verbose", C.c_int32),
                ("display_frequency", C.c_int32), ("use_graph", C.c_int32),
                ("timing_chunk", C.c_int32), ("eps_primal_infeasible", C.c_double),
                ("eps_dual_infeasible", C.c_double), ("feasibility_polishing", C.c_int32),
                ("eps_feas_polish", C.c_double), ("panel_rows", C.c_int32),
                ("panel_min_len", C.c_int32), ("panel_wgs", C.c_int32), ("hot_cols", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int64), ("restarts", C.c_int64),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double),
                ("rel_primal_res", C.c_double), ("rel_dual_res", C.c_double),
                ("rel_gap", C.c_double), ("kkt_rel", C.c_double),
                ("solve_seconds", C.c_double), ("setup_seconds", C.c_double),
                ("eta", C.c_double), ("omega", C.c_double), ("norm_a", C.c_double),
                ("norm_q", C.c_double), ("power_iters", C.c_int32),
                ("kernel_samples", C.c_int32), ("kernel_primal_ms", C.c_double),
                ("kernel_dual_ms", C.c_double), ("polish_iterations", C.c_int64)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class BatchProblem(C.Structure):
    _fields_ = [("batch", C.c_int32), ("shared_a", C.c_int32), ("m", C.c_int32), ("n", C.c_int32),
                ("a_rowptr", P), ("a_colidx", P), ("a_val", P), ("a_nnz", C.c_int64),
                ("row_off", P), ("col_off", P),
                ("c", P), ("lc", P), ("uc", P), ("lv", P), ("uv", P),
                ("q_rank", C.c_int32), ("q_factor", P), ("q_diag", P), ("mem", C.c_int32)]


# every symbol include/pdhg.h declares, with its ctypes signature
SIGNATURES = {
    "pdhg_options_default": (None, [C.POINTER(Options)]),
    "pdhg_last_error": (C.c_char_p, []),
    "pdhg_version": (C.c_int32, []),
    "pdhg_create": (C.c_int, [C.POINTER(Problem), C.POINTER(Options), P, C.POINTER(P)]),
    "pdhg_solve": (C.c_int, [P, P, P, P, P, C.POINTER(Result)]),
    "pdhg_update_data": (C.c_int, [P, P, P, P, P, P]),
    "pdhg_debug_step": (C.c_int, [P, P, P, P, P, C.c_int64, C.c_double, C.c_double, P, P, P, P]),
    "pdhg_debug_plain_step": (C.c_int, [P, P, P, P, P, C.c_int64, C.c_double, C.c_double, P, P]),
    "pdhg_get_scaling": (C.c_int, [P, P, P, P, P]),
    "pdhg_debug_qp_step": (C.c_int, [P, P, P, P, P, C.c_int64, C.c_double, P, P, P, P]),
    "pdhg_destroy": (None, [P]),
    "pdhg_batch_create": (C.c_int, [C.POINTER(BatchProblem), C.POINTER(Options), P, C.POINTER(P)]),
    "pdhg_batch_solve": (C.c_int, [P, P, P, P, P, P]),
    "pdhg_batch_set_launch": (C.c_int, [P, C.c_int32, C.c_int32]),
    "pdhg_batch_autotune": (C.c_int, [P, C.c_int32, C.POINTER(C.c_int32)]),
    "pdhg_batch_update_data": (C.c_int, [P, P, P, P, P, P]),
    "pdhg_batch_unrolled_forward": (C.c_int, [P, C.c_int64, C.c_int32, P, P]),
    "pdhg_batch_unrolled_backward": (C.c_int, [P, P, P, P, P, P, P]),
    "pdhg_linear_costs": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, P, P, P, P]),
    "pdhg_regret": (C.c_int, [C.c_int32, C.c_int32, P, P, P, P, P]),
    "pdhg_linear_costs_backward": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, P, P, P, P]),
    "pdhg_linear_costs_backward_noalloc": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, P, P, P, P]),
    "pdhg_qp_value": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P, P]),
    "pdhg_spo_plus_costs": (C.c_int, [C.c_int32, C.c_int32, P, P, P, P]),
    "pdhg_spo_plus": (C.c_int, [C.c_int32, C.c_int32, P, P, P, P, P, P, P, P]),
    "pdhg_pfy_costs": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, P, P, C.c_double, P, P]),
    "pdhg_pfy": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, P, P, P, C.c_double, P, P, P, P]),
    "pdhg_batch_destroy": (None, [P]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """Load the in-tree libpdhg.so; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise LibraryMissing(
                f"{LIB} is not built; run `python -m paper_2412_09734_amd._build` "
                "or __graft_entry__.build() first")
        L = C.CDLL(LIB)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class PdhgError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().pdhg_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({code}): {msg}")
        self.code = code


def check(code: int, where: str):
    if code != PDHG_OK:
        raise PdhgError(code, where)
