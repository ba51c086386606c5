"""MI355X-native randomized Tucker-sketched GMRES (HIP, gfx950).

The numerical work lives in ``libtsgmres.so`` (C ABI in ``include/tsgmres.h``);
this package is the thin Python binding.  Importing it does not load the
library; the first call does, and fails loudly if the library is not built.
"""
from ._abi import EXPORTS, LIB_PATH, TkError, load
from .api import (KronOp, MlnParams, SolveParams, Tucker, TuckerSGMRESLoss, apply_op, backward, kernel_timer,
                  kernel_timer_read, launch_count, launch_latency, rank_cert_count, mln_recover, mln_sketch, mln_solve, mln_solve_workspace_bytes, norm,
                  precond_tensors, project_core, projected_tikhonov, rhosvd, sketch, sketch_noalloc, solve, solve_workspace_bytes, storage_floats)

__all__ = ["EXPORTS", "LIB_PATH", "TkError", "load", "KronOp", "SolveParams", "Tucker", "TuckerSGMRESLoss",
           "apply_op", "backward", "kernel_timer", "kernel_timer_read", "launch_count", "launch_latency", "rank_cert_count", "norm", "rhosvd", "sketch", "sketch_noalloc", "solve",
           "solve_workspace_bytes", "storage_floats", "MlnParams", "mln_sketch", "mln_recover", "mln_solve",
           "mln_solve_workspace_bytes", "precond_tensors", "project_core", "projected_tikhonov"]
