"""MLN-Tucker sGMRES (Sec. 3.3: MLN_Sketch, MLN_Sum, MLN_Recovery and the
solver algorithm built on them) -- oracle, test infrastructure only.

Multilinear Nystrom approximation of a block sum ``sum_j c_j X^(j)`` with
Gaussian sketches Psi_k (n_k x r~, r~ = r + p) and the Khatri-Rao right
sketches Omega_k built from the leading r columns of the other modes' Psi:

  MLN_Sketch (per summand j):
      U_Psi_k = Psi_k^T U_k                      (r~ x r_k)
      Ubar_k  = first r rows of U_Psi_k          (r x r_k)
      G_Psi   = G x_1 U_Psi_1 ... x_d U_Psi_d    (r~^d)
      F_k     = U_k MTTKRP(G, {Ubar_l}, k)       (n_k x r)
  MLN_Sum:      G_Psi = sum_j c_j G_Psi^(j),  F_k = sum_j c_j F_k^(j)
  MLN_Recovery: Q_k R_k = qr(Psi_k^T F_k) (economy),  U~_k = F_k R_k^+,
                G~ = G_Psi x_1 Q_1^T ... x_d Q_d^T
  optional output of MLN_Sketch: diag(G_Psi), the superdiagonal of the
  summed sketched core, which equals the Khatri-Rao sketch
  (Psi_1 (.) ... (.) Psi_d)^T vec(sum_j c_j X^(j)) and serves as the sketch of
  the least-squares problem.

Readings where the paper leaves a choice (both sides use them):
  * Psi_k has r + p columns (the text; the solver listing writes n_k x r).
  * R_k^+ is the Moore-Penrose pseudoinverse with singular values at or
    below ``rcond * sigma_max`` treated as zero (rcond = 1e-12): in the first
    iterations the summed factors have rank below r and R_k is singular.
  * b_s = diag(G_Psi(B)) = beta diag(G_Psi(V_1)).
  * The window subtraction acts on the sketches (MLN_Sum); W is recovered
    again from the updated sketches before its norm is taken, so that
    V_{i+1} = W / ||W|| is the tensor whose sketches are stored.
  * All window coefficients h_{j,i} = <V_j, W> use the same recovered W
    (classical Gram-Schmidt, as in Alg. 2).
  * Breakdown when ||W|| <= 1e-14 ||W before the subtraction||, or when the
    new diagonal of the least-squares R is <= 1e-14 ||M||_F.
  * Norms of MLN outputs (whose factors are not orthonormal) are exact
    Frobenius norms of the Tucker tensor.
  * save_memory keeps the leading r~_sol = r_sol + p_sol indices of a stored
    sketched core and the leading r_sol columns of its factor sketches; the
    final recovery then uses the leading r~_sol columns of Psi_k.  The paper
    notes this equals sketching with those leading columns from the start.
  * Flexible preconditioning: Z_k is the MLN truncation of M(V_k), i.e.
    MLN_Recovery(MLN_Sketch of the 2q + 1 exponential-sum terms) with the
    same Psi and target rank r as every other sketch; the operator acts on
    that recovered Z_k, and its sketch (not V_k's) enters the final sum.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence

import numpy as np

from .roundsum import _mttkrp
from .sgmres import BREAKDOWN, NOT_CONVERGED, OK, sketched_lstsq
from .tikhonov import projected_tikhonov
from .tucker import Tucker, apply_op, exact_norm, inner, multi_ttm, scale

RCOND = 1e-12


@dataclasses.dataclass
class MLNSketch:
    """Sketched representation of a (sum of) Tucker tensor(s)."""
    core: np.ndarray        # G_Psi, r~^d
    F: List[np.ndarray]     # F_k, n_k x r


def mln_sketch(blocks, Psi: Sequence[np.ndarray], r: int):
    """MLN_Sketch of a block sum, summed with its coefficients (MLN_Sketch of
    every summand followed by MLN_Sum); returns (sketch, diag(G_Psi))."""
    d = blocks[0][1].d
    rt = Psi[0].shape[1]
    core = np.zeros((rt,) * d)
    F = [np.zeros((Pk.shape[0], r)) for Pk in Psi]
    for c, X in blocks:
        UPsi = [Pk.T @ Uk for Pk, Uk in zip(Psi, X.U)]          # r~ x r_k
        Ubar = [u[:r, :] for u in UPsi]                         # r x r_k
        core += c * multi_ttm(X.core, UPsi)
        for k in range(d):
            T = _mttkrp(X.core, [u.T for u in Ubar], k)         # r_k x r
            F[k] += c * (X.U[k] @ T)
    diag = np.array([core[(i,) * d] for i in range(rt)])
    return MLNSketch(core, F), diag


def mln_sum(sketches: Sequence[MLNSketch], coefs: Sequence[float]) -> MLNSketch:
    """MLN_Sum: linear combination of sketched cores and factor sketches."""
    core = sum(c * s.core for c, s in zip(coefs, sketches))
    F = [sum(c * s.F[k] for c, s in zip(coefs, sketches)) for k in range(len(sketches[0].F))]
    return MLNSketch(core, F)


def mln_recovery(sk: MLNSketch, Psi: Sequence[np.ndarray]) -> Tucker:
    """MLN_Recovery: economy QR of Psi_k^T F_k, factors F_k R_k^+, core
    G_Psi x_k Q_k^T."""
    Qs, Us = [], []
    for Pk, Fk in zip(Psi, sk.F):
        Q, R = np.linalg.qr(Pk.T @ Fk, mode="reduced")
        Us.append(Fk @ np.linalg.pinv(R, rcond=RCOND))
        Qs.append(Q.T)
    return Tucker(multi_ttm(sk.core, Qs), Us)


def truncate_sketch(sk: MLNSketch, rt_sol: int, r_sol: int) -> MLNSketch:
    """The memory-efficient truncation of a stored sketch (leading indices)."""
    d = sk.core.ndim
    return MLNSketch(sk.core[(slice(0, rt_sol),) * d].copy(), [F[:, :r_sol].copy() for F in sk.F])


@dataclasses.dataclass
class MLNParams:
    r: int = 32
    p: int = 32
    tol: float = 1e-8
    eta: float = 0.4
    maxiter: int = 60
    k_trunc: int = 2
    breakdown_tol: float = 1e-14
    save_memory: bool = False
    r_sol: int = 0
    p_sol: int = 0
    tikhonov: bool = False      # projected Tikhonov with GCV on the sketched LS (Sec. 4.3)


def mln_sgmres(terms, B: Tucker, Psi: Sequence[np.ndarray], prm: MLNParams, transpose: bool = False,
               log: Optional[list] = None, precond: Optional[Callable[[Tucker], list]] = None):
    """MLN-Tucker sGMRES on ``L(X) = B``; returns (X, info).  ``Psi`` are the
    n_k x (r + p) sketches.

    ``precond`` (optional) maps a basis tensor V to the block list of M(V)
    (Sec. 3.4).  The method is then flexible: the truncated preconditioned
    tensor is Z_k = MLN_Recovery(MLN_Sketch(M(V_k))), the operator acts on
    Z_k, only the sketches of the Z_k are kept for the solution (truncated to
    the solution sketch size in the memory-efficient variant), and the
    solution is recovered from sum_i y_i sketch(Z_i)."""
    r = prm.r
    beta = exact_norm([(1.0, B)])
    V = [scale(B, 1.0 / beta)]
    sk_v, b_s = mln_sketch([(1.0, V[0])], Psi, r)
    b_s = beta * b_s
    beta_s = float(np.linalg.norm(b_s))
    stored: List[MLNSketch] = [sk_v]
    rt_sol = prm.r_sol + prm.p_sol
    cols: List[np.ndarray] = []
    hist: List[float] = []
    lams: List[float] = []
    zsk: List[MLNSketch] = []
    status = NOT_CONVERGED
    y = np.zeros(0)
    i = 0
    for i in range(1, prm.maxiter + 1):
        if precond is not None:
            skZ, _ = mln_sketch(precond(V[-1]), Psi, r)
            Z = mln_recovery(skZ, Psi)
            zsk.append(truncate_sketch(skZ, rt_sol, prm.r_sol) if prm.save_memory else skZ)
            LV = apply_op(terms, Z, transpose=transpose)
        else:
            LV = apply_op(terms, V[-1], transpose=transpose)
        skW, sW = mln_sketch(LV, Psi, r)
        cols.append(sW)
        W = mln_recovery(skW, Psi)
        wnorm = exact_norm([(1.0, W)])
        j0 = max(1, i - prm.k_trunc + 1)
        h = [inner(V[j - 1], W) for j in range(j0, i + 1)]
        skW = mln_sum([skW] + [stored[j - 1] for j in range(j0, i + 1)], [1.0] + [-hj for hj in h])
        W = mln_recovery(skW, Psi)
        omega = exact_norm([(1.0, W)])
        M = np.stack(cols, axis=1)
        y, res, rkk = sketched_lstsq(M, b_s)
        if prm.tikhonov:
            y, res, lam = projected_tikhonov(M, b_s)
            lams.append(lam)
        rel = res / beta_s
        hist.append(rel)
        if log is not None:
            log.append(dict(k=i, h=h, omega=omega, res=rel, ranks=W.ranks))
        if omega <= prm.breakdown_tol * wnorm or rkk <= prm.breakdown_tol * np.linalg.norm(M):
            status = BREAKDOWN
            break
        V.append(scale(W, 1.0 / omega))
        sk_next, _ = mln_sketch([(1.0, V[-1])], Psi, r)
        stored.append(sk_next)
        if i > prm.k_trunc:
            V[i - prm.k_trunc - 1] = None      # outside the window: only its sketch is kept
            if prm.save_memory:
                stored[i - prm.k_trunc - 1] = truncate_sketch(stored[i - prm.k_trunc - 1], rt_sol, prm.r_sol)
        if rel < prm.eta * prm.tol:
            status = OK
            break
    n_used = len(y)
    final_sk = (zsk if precond is not None else stored)[:n_used]
    Psi_rec = Psi
    if prm.save_memory:
        final_sk = [s if s.core.shape[0] == rt_sol else truncate_sketch(s, rt_sol, prm.r_sol) for s in final_sk]
        Psi_rec = [Pk[:, :rt_sol] for Pk in Psi]
    X = mln_recovery(mln_sum(final_sk, [float(v) for v in y]), Psi_rec)
    Bn = exact_norm([(1.0, B)])
    true_res = exact_norm([(1.0, B)] + [(-c, T) for c, T in apply_op(terms, X, transpose=transpose)]) / Bn
    return X, dict(status=status, iters=i, hist=hist, true_relres=true_res, beta=beta, beta_s=beta_s,
                   lam=lams)
