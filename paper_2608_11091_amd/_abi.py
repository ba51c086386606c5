"""ctypes mirror of ``include/tsgmres.h`` and the library loader.

The loader never falls back to anything: if ``libtsgmres.so`` is missing or
does not load, it raises.  Building happens only through
``paper_2608_11091_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as C
import os

TK_MAX_D = 4
HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsgmres.so")

STATUS = {0: "ok", 1: "not_converged", 2: "breakdown", 3: "rank_floor"}
ERRORS = {-1: "invalid argument", -2: "shape", -3: "capacity", -4: "workspace", -5: "hip",
          -6: "non-finite", -7: "unsupported"}

# the structures below mirror include/tsgmres.h at this ABI version
ABI_VERSION = 205

EXPORTS = [
    "tucker_apply_op", "tucker_apply_op_workspace", "tucker_sketch", "tucker_sketch_workspace",
    "tucker_sketch_noalloc",
    "tucker_rhosvd", "tucker_rhosvd_workspace", "tsgmres_solve", "tsgmres_solve_workspace",
    "tsgmres_backward", "tsgmres_backward_workspace", "tucker_norm", "tucker_norm_workspace",
    "tucker_mln_sketch", "tucker_mln_sketch_workspace", "tucker_mln_recover", "tucker_mln_recover_workspace",
    "tsgmres_mln_solve", "tsgmres_mln_solve_workspace",
    "tsgmres_projected_tikhonov", "tsgmres_projected_tikhonov_workspace",
    "tk_kernel_timer", "tk_kernel_timer_read", "tk_launch_count", "tk_launch_latency", "tk_rank_cert_count",
    "tk_last_error", "tk_version",
]


class TkTucker(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int64 * TK_MAX_D), ("r", C.c_int64 * TK_MAX_D),
                ("rcap", C.c_int64 * TK_MAX_D), ("core", C.c_void_p), ("U", C.c_void_p * TK_MAX_D)]


class TkBlockSum(C.Structure):
    _fields_ = [("nblocks", C.c_int32), ("coef", C.POINTER(C.c_double)), ("blocks", C.POINTER(TkTucker))]


class TkKronOp(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int64 * TK_MAX_D), ("nterms", C.c_int32),
                ("alpha", C.POINTER(C.c_double)), ("A", C.POINTER(C.c_void_p))]


class TkRoundParams(C.Structure):
    _fields_ = [("eps", C.c_double), ("tau", C.c_double), ("rank_cap", C.c_int32), ("oversample", C.c_int32),
                ("force_s", C.c_int32), ("force_ranks", C.c_int32 * TK_MAX_D), ("form", C.c_int32)]


class TkSgmresParams(C.Structure):
    _fields_ = [("form", C.c_int32), ("tol", C.c_double), ("eta", C.c_double), ("maxiter", C.c_int32),
                ("max_restarts", C.c_int32), ("k_trunc", C.c_int32), ("rank_cap", C.c_int32),
                ("oversample", C.c_int32), ("s", C.c_int64), ("eps_trunc", C.c_double), ("eps_min", C.c_double),
                ("tol_inner_floor", C.c_double), ("x0", C.POINTER(TkTucker)), ("precond_q", C.c_int32),
                ("precond_V", C.POINTER(C.c_void_p)), ("precond_lambda", C.POINTER(C.c_void_p)),
                ("tikhonov", C.c_int32), ("method", C.c_int32)]


class TkMlnParams(C.Structure):
    _fields_ = [("r", C.c_int32), ("p", C.c_int32), ("tol", C.c_double), ("eta", C.c_double),
                ("maxiter", C.c_int32), ("k_trunc", C.c_int32), ("breakdown_tol", C.c_double),
                ("save_memory", C.c_int32), ("r_sol", C.c_int32), ("p_sol", C.c_int32),
                ("tikhonov", C.c_int32), ("precond_q", C.c_int32), ("precond_V", C.POINTER(C.c_void_p)),
                ("precond_lambda", C.POINTER(C.c_void_p))]


class TkSgmresInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters_total", C.c_int32), ("cycles", C.c_int32),
                ("true_relres", C.c_double), ("seconds", C.c_double), ("hist_cap", C.c_int32),
                ("hist_len", C.c_int32), ("hist_sketched", C.POINTER(C.c_double)),
                ("hist_true", C.POINTER(C.c_double)), ("hist_ranks", C.POINTER(C.c_int32)),
                ("hist_cycle_seconds", C.POINTER(C.c_double)), ("hist_lambda", C.POINTER(C.c_double))]


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Loads the HIP library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2608_11091_amd.build`")
    lib = C.CDLL(path)
    P, VP, SZ = C.POINTER, C.c_void_p, C.c_size_t
    lib.tucker_apply_op.argtypes = [P(TkKronOp), P(TkTucker), C.c_int32, C.c_int32, P(VP), VP, SZ, VP]
    lib.tucker_apply_op_workspace.argtypes = [P(TkKronOp), P(TkTucker), C.c_int32, P(SZ)]
    lib.tucker_sketch.argtypes = [P(TkBlockSum), P(VP), C.c_int64, C.c_int32, VP, VP, SZ, VP]
    lib.tucker_sketch_workspace.argtypes = [P(TkBlockSum), C.c_int64, C.c_int32, P(SZ)]
    lib.tucker_sketch_noalloc.argtypes = [P(TkBlockSum), P(VP), C.c_int64, C.c_int32, VP, VP]
    lib.tucker_rhosvd.argtypes = [P(TkBlockSum), P(TkRoundParams), P(VP), P(TkTucker), P(C.c_int32), VP, SZ, VP]
    lib.tucker_rhosvd_workspace.argtypes = [P(TkBlockSum), P(TkRoundParams), P(SZ)]
    lib.tsgmres_solve.argtypes = [P(TkKronOp), P(TkTucker), P(TkSgmresParams), P(VP), P(VP), P(TkTucker),
                                  P(TkSgmresInfo), VP, SZ, VP]
    lib.tsgmres_solve_workspace.argtypes = [P(TkKronOp), P(TkTucker), P(TkSgmresParams), P(SZ)]
    lib.tsgmres_backward.argtypes = [P(TkKronOp), P(TkTucker), P(TkBlockSum), P(TkSgmresParams), P(VP), P(VP),
                                     P(TkTucker), P(C.c_double), P(VP), P(TkSgmresInfo), VP, SZ, VP]
    lib.tsgmres_backward_workspace.argtypes = [P(TkKronOp), P(TkTucker), P(TkBlockSum), P(TkSgmresParams), P(SZ)]
    lib.tucker_norm.argtypes = [P(TkBlockSum), P(C.c_double), VP, SZ, VP]
    lib.tucker_norm_workspace.argtypes = [P(TkBlockSum), P(SZ)]
    I32, I64 = C.c_int32, C.c_int64
    lib.tucker_mln_sketch.argtypes = [P(TkBlockSum), P(VP), I32, I32, VP, P(VP), VP, VP, SZ, VP]
    lib.tucker_mln_sketch_workspace.argtypes = [P(TkBlockSum), I32, I32, P(SZ)]
    lib.tucker_mln_recover.argtypes = [VP, P(VP), P(VP), I32, I32, P(TkTucker), VP, SZ, VP]
    lib.tucker_mln_recover_workspace.argtypes = [I32, P(I64), I32, I32, P(SZ)]
    lib.tsgmres_mln_solve.argtypes = [P(TkKronOp), P(TkTucker), P(TkMlnParams), P(VP), P(TkTucker),
                                      P(TkSgmresInfo), VP, SZ, VP]
    lib.tsgmres_mln_solve_workspace.argtypes = [P(TkKronOp), P(TkTucker), P(TkMlnParams), P(SZ)]
    lib.tsgmres_projected_tikhonov.argtypes = [VP, VP, I32, I32, C.c_double, VP, VP, VP, SZ, VP]
    lib.tsgmres_projected_tikhonov_workspace.argtypes = [I32, I32, P(SZ)]
    lib.tk_kernel_timer.argtypes = [C.c_int32, C.c_int32]
    lib.tk_kernel_timer_read.argtypes = [C.c_int32, P(C.c_int64), P(C.c_double), P(C.c_double), P(C.c_double)]
    lib.tk_launch_count.argtypes = [C.POINTER(C.c_int64)]
    lib.tk_launch_latency.argtypes = [C.c_int32, C.c_void_p, C.POINTER(C.c_double)]
    lib.tk_rank_cert_count.argtypes = [C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.tk_last_error.restype = C.c_char_p
    lib.tk_version.restype = C.c_int
    for name in EXPORTS:
        if not hasattr(lib, name):
            raise RuntimeError(f"{path} does not export {name}")
    if lib.tk_version() != ABI_VERSION:
        raise RuntimeError(f"{path} has ABI version {lib.tk_version()}, the binding expects {ABI_VERSION}: rebuild")
    _lib = lib
    return lib


class TkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tsgmres error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


def check(code: int) -> int:
    if code < 0:
        raise TkError(code, load().tk_last_error().decode())
    return code
