"""ctypes view of the C ABI declared in include/pgdto.h (argument marshalling only).

Every computation happens in the HIP library ``libpgdto.so`` built in-tree by
``build.py``.  If the library is missing this module raises ImportError: there
is no Python or CPU fallback for the projection.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PGDTO_LIB selects another build of the same library (the sanitizer build,
# libpgdto_san.so, for the CPU test suite)
LIB_PATH = os.environ.get("PGDTO_LIB") or os.path.join(HERE, "libpgdto.so")

MAX_M = 64          # coupled rows (beyond SMALL_M: float32 projections, one-instance launches)
SMALL_M = 8
MAX_BLOCKS = 64

# enums (pgdto.h)
OK, PENDING, QUEUED = 0, 1, 2
ERR_ARG, ERR_HIP, ERR_NOMEM, ERR_UNKNOWN_TICKET, ERR_TIMEOUT, ERR_BUSY, ERR_CANCELLED, ERR_SCRATCH = (
    -1, -2, -3, -4, -5, -6, -7, -8)
NOALLOC_SCRATCH_BYTES = 1466752
BATCH_MAX = 256
CONVERGED, INACTIVE, INFEASIBLE, MAXITER, NONFINITE = 0, 1, 2, 3, 4
OUTCOME_NAMES = {0: "converged", 1: "inactive", 2: "infeasible", 3: "maxiter", 4: "nonfinite"}
F32, F64 = 0, 1
SINGLE, INDEPENDENT, COUPLED = 0, 1, 2
KINDS = {"single": SINGLE, "independent": INDEPENDENT, "coupled": COUPLED}
SEARCH_NEWTON, SEARCH_BISECT = 0, 1
NCP_CONTINUOUS, NCP_PAPER = 0, 1
CG_PR_PLUS, CG_FR, CG_NONE = 0, 1, 2
CG_RULES = {"pr+": CG_PR_PLUS, "fr": CG_FR, "none": CG_NONE}


class Problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("n", C.c_int64), ("m", C.c_int32),
                ("y", C.c_void_p), ("A", C.c_void_p), ("lda", C.c_int64),
                ("block_offsets", C.POINTER(C.c_int64)), ("b", C.POINTER(C.c_double)),
                ("lo", C.c_double), ("hi", C.c_double), ("C", C.c_double),
                ("x", C.c_void_p), ("free_mask", C.c_void_p), ("eq_mask", C.c_uint64),
                ("lambda0", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("tol_b", C.c_double), ("tol_n", C.c_double),
                ("max_search", C.c_int32), ("max_newton", C.c_int32), ("max_ls", C.c_int32),
                ("search", C.c_int32), ("ncp", C.c_int32), ("stage1", C.c_int32),
                ("c1", C.c_double), ("c2", C.c_double), ("compact", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("outcome", C.c_int32), ("path", C.c_int32), ("passes", C.c_int32),
                ("iters_search", C.c_int32), ("iters_newton", C.c_int32), ("iters_ls", C.c_int32),
                ("m", C.c_int32), ("error", C.c_int32), ("n_free", C.c_int64),
                ("lambda_", C.c_double * MAX_BLOCKS), ("resid", C.c_double * MAX_BLOCKS),
                ("slack", C.c_double * MAX_BLOCKS), ("row_outcome", C.c_int32 * MAX_BLOCKS),
                ("res_inf", C.c_double), ("lambda_width", C.c_double), ("kappa", C.c_double),
                ("lambda_err", C.c_double * MAX_BLOCKS), ("x_err", C.c_double), ("n_compact", C.c_int64),
                ("passes_compacted", C.c_int32), ("reserved", C.c_int32), ("dist2", C.c_double)]

    def to_dict(self) -> dict:
        m = self.m
        return {"outcome": OUTCOME_NAMES.get(self.outcome, str(self.outcome)),
                "path": self.path, "passes": self.passes, "iters_search": self.iters_search,
                "iters_newton": self.iters_newton, "iters_ls": self.iters_ls, "m": m,
                "error": self.error, "n_free": self.n_free,
                "lam": list(self.lambda_[:m]), "resid": list(self.resid[:m]),
                "slack": list(self.slack[:m]),
                "row_outcome": [OUTCOME_NAMES.get(o, str(o)) for o in self.row_outcome[:m]],
                "res_inf": self.res_inf, "lambda_width": self.lambda_width, "kappa": self.kappa,
                "lambda_err": list(self.lambda_err[:m]), "x_err": self.x_err, "n_compact": self.n_compact,
                "passes_compacted": self.passes_compacted, "dist2": self.dist2}


class PgdArgs(C.Structure):
    _fields_ = [("proj", Problem), ("rho", C.c_void_p), ("rho_prev", C.c_void_p),
                ("grad", C.c_void_p), ("grad_prev", C.c_void_p), ("dir", C.c_void_p),
                ("g", C.POINTER(C.c_double)), ("G", C.POINTER(C.c_double)), ("t", C.c_int64),
                ("t_warmup", C.c_int32), ("cg_rule", C.c_int32),
                ("alpha_max", C.c_double), ("alpha_fallback", C.c_double), ("omega", C.c_double),
                ("eps_alpha", C.c_double), ("tol_viol", C.c_double), ("tol", C.c_double),
                ("work", C.c_void_p)]


class PgdOut(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta", C.c_double), ("rel_change", C.c_double),
                ("used_fallback", C.c_int32), ("converged", C.c_int32), ("proj", Result)]

    def to_dict(self) -> dict:
        return {"alpha": self.alpha, "beta": self.beta, "rel_change": self.rel_change,
                "used_fallback": bool(self.used_fallback), "converged": bool(self.converged),
                "proj": self.proj.to_dict()}


class BatchCfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("wg_per_slot", C.c_int32), ("queue_capacity", C.c_int32), ("slots_only", C.c_int32)]


class PathPoint(C.Structure):
    _fields_ = [("C", C.c_double), ("kappa", C.c_double), ("dist", C.c_double), ("max_violation", C.c_double),
                ("violation_over_tau", C.c_double), ("outcome", C.c_int32), ("passes", C.c_int32),
                ("lambda_", C.c_double * MAX_BLOCKS), ("slack", C.c_double * MAX_BLOCKS),
                ("violation", C.c_double * MAX_BLOCKS)]

    def to_dict(self, m: int) -> dict:
        return {"C": self.C, "kappa": self.kappa, "dist": self.dist, "max_violation": self.max_violation,
                "violation_over_tau": self.violation_over_tau,
                "outcome": OUTCOME_NAMES.get(self.outcome, str(self.outcome)), "passes": self.passes,
                "lam": list(self.lambda_[:m]), "slack": list(self.slack[:m]), "violation": list(self.violation[:m])}


STRUCTS = [Problem, Params, Result, PgdArgs, PgdOut, BatchCfg, PathPoint]

# every function the header declares: name -> (restype, argtypes)
_VP = C.c_void_p
SIGNATURES = {
    "pgdto_params_default": (None, [C.POINTER(Params)]),
    "pgdto_pgd_args_default": (None, [C.POINTER(PgdArgs)]),
    "pgdto_ctx_create": (C.c_int, [C.c_int, C.POINTER(_VP)]),
    "pgdto_ctx_destroy": (C.c_int, [_VP]),
    "pgdto_ctx_autotune": (C.c_int, [_VP, C.c_int]),
    "pgdto_ctx_last_launch": (C.c_int, [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "pgdto_ctx_autotune_save": (C.c_int, [_VP, C.c_char_p]),
    "pgdto_ctx_autotune_load": (C.c_int, [_VP, C.c_char_p]),
    "pgdto_project": (C.c_int, [_VP, C.POINTER(Problem), C.POINTER(Params), C.POINTER(Result), _VP]),
    "pgdto_project_async": (C.c_int, [_VP, C.POINTER(Problem), C.POINTER(Params), _VP, _VP]),
    "pgdto_project_noalloc": (C.c_int, [C.POINTER(Problem), C.POINTER(Params), _VP, _VP]),
    "pgdto_pgd_step": (C.c_int, [_VP, C.POINTER(PgdArgs), C.POINTER(Params), C.POINTER(PgdOut), _VP]),
    "pgdto_pgd_step_async": (C.c_int, [_VP, C.POINTER(PgdArgs), C.POINTER(Params), _VP, _VP]),
    "pgdto_project_batch_async": (C.c_int, [_VP, C.POINTER(Problem), C.c_int, C.POINTER(Params), _VP, C.c_int, _VP]),
    "pgdto_pgd_step_batch_async": (C.c_int, [_VP, C.POINTER(PgdArgs), C.c_int, C.POINTER(Params), _VP, C.c_int,
                                             _VP]),
    "pgdto_batch_create": (C.c_int, [_VP, C.POINTER(BatchCfg), C.POINTER(_VP)]),
    "pgdto_batch_submit": (C.c_int, [_VP, C.POINTER(Problem), C.POINTER(Params), C.POINTER(C.c_uint64)]),
    "pgdto_batch_poll": (C.c_int, [_VP, C.c_uint64, C.POINTER(Result)]),
    "pgdto_batch_wait": (C.c_int, [_VP, C.c_uint64, C.POINTER(Result)]),
    "pgdto_batch_poll_timed": (C.c_int, [_VP, C.c_uint64, C.POINTER(Result), C.POINTER(C.c_int64), C.c_int]),
    "pgdto_batch_submit_pgd": (C.c_int, [_VP, C.POINTER(PgdArgs), C.POINTER(Params), C.POINTER(C.c_uint64)]),
    "pgdto_batch_poll_pgd": (C.c_int, [_VP, C.c_uint64, C.POINTER(PgdOut), C.POINTER(C.c_int64), C.c_int]),
    "pgdto_batch_shape": (C.c_int, [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "pgdto_batch_stats": (C.c_int, [_VP] + [C.POINTER(C.c_int64)] * 5),
    "pgdto_batch_autotune": (C.c_int, [_VP, C.POINTER(Problem), C.c_int, C.POINTER(Params), C.c_int,
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "pgdto_batch_destroy": (C.c_int, [_VP]),
    "pgdto_status_string": (C.c_char_p, [C.c_int]),
    "pgdto_version": (C.c_int, []),
    "pgdto_problem_check": (C.c_int, [C.POINTER(Problem), C.POINTER(Params)]),
    "pgdto_struct_size": (C.c_size_t, [C.c_int]),
    "pgdto_trace_read": (C.c_int, [_VP, C.POINTER(C.c_uint64), C.c_int]),
    "pgdto_kappa_path": (C.c_int, [_VP, C.POINTER(Problem), C.POINTER(Params), C.POINTER(C.c_double), C.c_int,
                                   C.c_double, C.POINTER(PathPoint), _VP]),
}

_lib = None


def lib():
    """Load libpgdto.so (built in-tree); raise if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "or `python paper_2511_13905_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    for i, S in enumerate(STRUCTS):
        got = L.pgdto_struct_size(i)
        if got != C.sizeof(S):
            raise ImportError(f"ABI mismatch for {S.__name__}: C {got} bytes, ctypes {C.sizeof(S)}")
    _lib = L
    return L


def status_string(st: int) -> str:
    return lib().pgdto_status_string(st).decode()


class PgdtoError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status
