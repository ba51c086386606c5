"""Plain FP64 CPU oracle of randomized Tucker-sketched GMRES.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_2608_11091_amd``); the two meet only through the seeded
inputs of ``workloads``.

Every routine is written for a reader checking it against the paper by eye:
NumPy/SciPy library primitives (tensordot, Householder QR, SVD, symmetric
eigenvalues) serve as steps, with no blocking, fusion or reordering beyond
what the paper's definitions state.

Parity status (see the pins in ``tests/test_oracle_*.py``):
  * apply / sketch / inner / exact norm: pinned (dense brute force, closed
    forms, the superdiagonal identity of Sec. 3.3).
  * RoundSum: pinned (exactness at eps=0, energy identity, error bound,
    truncated HOSVD of the dense sum).
  * sGMRES cycle / restarted solve: pinned (textbook GMRES reduction,
    residual identity, exact solutions).
  * adjoint gradients: pinned (dense gradient, finite differences).
  * MLN-Tucker sGMRES (``oracle.mln``): pinned (dense sketches and the
    Khatri-Rao identity, Nystrom exactness below the target rank, the
    memory-efficient truncation identity, reduction to vector sketched GMRES
    when the recovery is exact, a tiny Poisson solve).
  * exponential-sum preconditioner and flexible cycle (``oracle.precond``):
    pinned (closed-form DST-I eigenpairs of the 1D Laplacian, the
    exponential sum's relative error against 1/x over the spectrum, the
    spectral application against the dense sum of matrix exponentials and
    against the dense inverse, and the flexible cycle against the dense
    solution).
  * RHOSVD-Tucker GMRES, full Arnoldi (``oracle.gmres``): pinned (dense
    textbook GMRES with exact RoundSums, the Arnoldi relation and
    orthonormality of the basis, the Poisson closed form, lucky breakdown on
    an eigentensor).
  * projected Tikhonov with GCV (``oracle.tikhonov``): pinned (the stacked
    least-squares solution, the influence-matrix definition of GCV, the
    closed-form minimiser for equal singular values, brute-force
    minimisation on a fine grid, the lambda -> 0 limit, and the removal of
    semiconvergence on a noisy blur problem).
  * effective-rank heuristic (Sec. 3.1): pinned (the threshold and the
    |c| ||G|| weighting on a constructed sum whose Gram tail sits just above
    and just below tau^2 sum(lambda); the numerical rank of a wide
    concatenation counted from its SVD; invariance under splitting a summand
    and under a global scale).  Whether the width it picks gives a good
    range sketch is probabilistic and stays unpinned.
"""
from .tucker import (Tucker, to_dense, ttm, multi_ttm, unfold, apply_op, transpose_terms,
                     dense_operator, sketch_krp, sketch_kron, inner, exact_norm,
                     block_dense, scale)
from .roundsum import RoundParams, roundsum, effective_sketch_size, st_hosvd
from .sgmres import SGMRESParams, sgmres_cycle, solve, sketched_lstsq
from .adjoint import adjoint_gradients, loss_and_cotangent
from . import gmres, mln, precond, tikhonov

__all__ = [
    "Tucker", "to_dense", "ttm", "multi_ttm", "unfold", "apply_op", "transpose_terms",
    "dense_operator", "sketch_krp", "sketch_kron", "inner", "exact_norm", "block_dense",
    "scale", "RoundParams", "roundsum", "effective_sketch_size", "st_hosvd",
    "SGMRESParams", "sgmres_cycle", "solve", "sketched_lstsq", "adjoint_gradients",
    "loss_and_cotangent", "gmres", "mln", "precond", "tikhonov",
]
