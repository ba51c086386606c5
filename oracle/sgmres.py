"""RHOSVD-Tucker sGMRES (Alg. 2) with restarts and FP64 iterative
refinement -- oracle, test infrastructure only.

Alg. 2 step by step (one cycle, ``sgmres_cycle``):
  beta = ||B||, V_1 = B / beta, b_s = S^T vec(B), beta_s = ||b_s||;
  for k = 1..N_max:
      W = RoundSum(L(V_k))                     (operator apply + recompression)
      M = [M, S^T vec(W)]                      (sketch of the rounded W)
      W = RoundSum(W - sum_{window} <V_j, W> V_j)   (truncated Arnoldi, window k_trunc)
      y_k = argmin ||M y - b_s||, res_k = ||M y_k - b_s|| / beta_s
      if ||W|| ~ 0: stop (breakdown);  V_{k+1} = W / ||W||
      if res_k < eta * tol: stop
  X = RoundSum(sum_i y_i V_i)

Readings where the paper leaves a choice: classical one-pass orthogonalisation (all
coefficients from the same W, one RoundSum of 1 + window blocks); y_k is
computed before the breakdown test; breakdown when ||W|| <= 1e-14 ||RoundSum(L V_k)||
or the new diagonal of the least-squares R factor is <= 1e-14 ||M||_F; the
least squares use a Householder QR without pivoting.

Restarts (``solve``): the paper discourages restarting for memory reasons but
does not define it; the solver here wraps cycles in FP64 iterative refinement:
x_0 = 0, r_0 = B; per cycle solve L d = r_c to relative tolerance
``tol ||B|| / ||r_c||`` (floored), ``x <- RoundSum(x + d)``, then the exact FP64
residual ``||B - L(x)|| / ||B||`` (QR of concatenated factors) decides;
``r_{c+1} = RoundSum(B - L(x))``.  Two cycles in a row that reduce the true
residual by less than 10% stop the solve with a rank-floor status.  A solve
that stops without converging returns the iterate with the smallest true
residual (cycles on a rank floor can raise it: x + d is rounded back to the
rank cap).  A floor reached while every rank of x is below the cap comes
from the update's truncation tolerance (on an operator of condition number
kappa, rounding x + d to relative accuracy eps moves the residual by up to
about kappa eps): the tolerance is then divided by 100, down to 1e-15, and
the refinement goes on, with the floor test counting cycles afresh.  These
outer RoundSums use the full sketch width cap + p: the effective-rank rule of
Sec. 3.1 sizes the sketch from the weighted factor Gram, where a correction d
far smaller than x (or a residual far smaller than B and L(x)) sits below the
Gram's rounding level and would be left to the p oversampling columns.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional

import numpy as np
from scipy.linalg import solve_triangular

from .roundsum import RoundParams, roundsum
from .tikhonov import projected_tikhonov
from .tucker import Tucker, apply_op, exact_norm, inner, scale, sketch_krp

OK, NOT_CONVERGED, BREAKDOWN, RANK_FLOOR = 0, 1, 2, 3
EPS_OUTER_MIN = 1e-15


@dataclasses.dataclass
class SGMRESParams:
    tol: float = 1e-8
    eta: float = 0.4
    maxiter: int = 60
    k_trunc: int = 2
    max_restarts: int = 50
    cap: int = 48
    p: int = 5
    eps_trunc: Optional[float] = None      # inner RoundSums (default 1e-2 * inner tol)
    eps_min: float = 1e-13                 # floor of the inner truncation tolerance
    tol_inner_floor: float = 1e-13         # floor of the per-cycle relative tolerance
    eps_outer: Optional[float] = None      # x-update / residual RoundSums (default 1e-2 * tol)
    breakdown_tol: float = 1e-14
    replay: Optional[dict] = None          # rank replay: {"s": [...], "ranks": [...]} consumed in order
    range_basis: Optional[Callable] = None  # basis routine of the cycle's RoundSums (None: Householder)
    operand_rounding: Optional[Callable] = None  # rounding of the cycle's RoundSum operands (None: none)
    tikhonov: bool = False                 # projected Tikhonov with GCV on the sketched LS (Sec. 4.3)


def sketched_lstsq(M: np.ndarray, b: np.ndarray):
    """Sketched least squares (Eq. for y_k of sGMRES): Householder QR of M,
    triangular solve, residual ``||M y - b||``.  Returns (y, res, |R_kk|)."""
    Q, R = np.linalg.qr(M, mode="reduced")
    y = solve_triangular(R, Q.T @ b)
    res = float(np.linalg.norm(M @ y - b))
    return y, res, float(abs(R[-1, -1]))


class _Replay:
    def __init__(self, rep):
        self.rep = rep
        self.i = 0

    def next(self, prm: RoundParams) -> RoundParams:
        if self.rep is None:
            return prm
        s = self.rep["s"][self.i]
        r = self.rep["ranks"][self.i]
        self.i += 1
        return dataclasses.replace(prm, force_s=s, force_ranks=r)


def sgmres_cycle(terms, B: Tucker, S, Omega, prm: SGMRESParams, tol: Optional[float] = None,
                 transpose: bool = False, log: Optional[list] = None, replay=None, precond=None):
    """One cycle of Alg. 2 on ``L(X) = B``; returns (X, info).

    ``precond`` (optional) makes the cycle flexible (Sec. 3.4): it maps
    (V_k, round_fn) to the preconditioned tensor Z_k = T(M(V_k)), where
    round_fn is the cycle's RoundSum; the operator is applied to Z_k and the
    solution is RoundSum(sum_i y_i Z_i)."""
    tol = prm.tol if tol is None else tol
    eps = prm.eps_trunc if prm.eps_trunc is not None else max(1e-2 * tol, prm.eps_min)
    rp = RoundParams(eps=eps, cap=prm.cap, p=prm.p, range_basis=prm.range_basis,
                     operand_rounding=prm.operand_rounding)
    rep = replay if replay is not None else _Replay(prm.replay)
    beta = exact_norm([(1.0, B)])
    V = [scale(B, 1.0 / beta)]
    b_s = sketch_krp([(1.0, B)], S)
    beta_s = float(np.linalg.norm(b_s))
    cols: List[np.ndarray] = []
    hist = []
    status = NOT_CONVERGED
    y = np.zeros(0)
    k = 0
    Z: List[Tucker] = []
    lams = []
    for k in range(1, prm.maxiter + 1):
        Zk = V[-1]
        if precond is not None:
            # the 2q + 1 terms of the preconditioner are rounded at the full sketch
            # width cap + p (their concatenated factors exceed the effective-rank rule)
            rpz = dataclasses.replace(rp, force_s=prm.cap + prm.p)
            Zk = precond(V[-1], lambda blocks: roundsum(blocks, Omega, rep.next(rpz))[0])
            Z.append(Zk)
        LV = apply_op(terms, Zk, transpose=transpose)
        W, i1 = roundsum(LV, Omega, rep.next(rp))
        cols.append(sketch_krp([(1.0, W)], S))
        window = V[max(0, k - prm.k_trunc):k]
        h = [inner(Vj, W) for Vj in window]
        W2, i2 = roundsum([(1.0, W)] + [(-hj, Vj) for hj, Vj in zip(h, window)], Omega, rep.next(rp))
        omega = float(np.linalg.norm(W2.core.ravel()))
        wnorm = float(np.linalg.norm(W.core.ravel()))
        M = np.stack(cols, axis=1)
        y, res, rkk = sketched_lstsq(M, b_s)
        if prm.tikhonov:
            # the regularised y_k replaces the least-squares one; the breakdown
            # test still reads the unregularised R factor
            y, res, lam = projected_tikhonov(M, b_s)
            lams.append(lam)
        rel = res / beta_s
        hist.append(rel)
        if log is not None:
            log.append(dict(k=k, s1=i1["s"], r1=i1["ranks"], s2=i2["s"], r2=i2["ranks"], h=h,
                            omega=omega, res=rel, lam=lams[-1] if lams else None))
        if omega <= prm.breakdown_tol * wnorm or rkk <= prm.breakdown_tol * np.linalg.norm(M):
            status = BREAKDOWN
            break
        V.append(scale(W2, 1.0 / omega))
        if rel < prm.eta * tol:
            status = OK
            break
    basis = Z if precond is not None else V
    X, i3 = roundsum([(float(y[i]), basis[i]) for i in range(len(y))], Omega, rep.next(rp))
    if log is not None:
        log.append(dict(final=True, s=i3["s"], r=i3["ranks"]))
    return X, dict(status=status, iters=k, hist=hist, beta=beta, beta_s=beta_s, lam=lams)


def _residual_blocks(terms, B: Tucker, X: Tucker, transpose=False):
    """Block sum of ``B - L(X)``."""
    return [(1.0, B)] + [(-c, T) for c, T in apply_op(terms, X, transpose=transpose)]


def solve(terms, B: Tucker, S, Omega, prm: SGMRESParams, transpose: bool = False,
          x0: Optional[Tucker] = None, log: Optional[list] = None, precond=None, method: str = "sgmres"):
    """Restarted Tucker sGMRES with FP64 iterative refinement.  ``method``
    "gmres" runs full-Arnoldi cycles (Alg. 1, ``oracle.gmres``) inside the same
    refinement loop; S is then unused."""
    t0 = time.perf_counter()
    eps_out = prm.eps_outer if prm.eps_outer is not None else 1e-2 * prm.tol
    rpo = RoundParams(eps=eps_out, cap=prm.cap, p=prm.p, force_s=prm.cap + prm.p)
    rep = _Replay(prm.replay)
    bnorm = exact_norm([(1.0, B)])
    if x0 is None:
        x = None
        r = B
        rnorm = bnorm
    else:
        x = x0
        Rb = _residual_blocks(terms, B, x, transpose)
        rnorm = exact_norm(Rb)
        r, _ = roundsum(Rb, Omega, rep.next(rpo))
    true_hist, iters, status = [], 0, NOT_CONVERGED
    cycles = 0
    floor_from = 0          # the floor test looks at cycles from this index on
    best = (rnorm, x) if x is not None else (np.inf, None)
    for c in range(prm.max_restarts):
        if rnorm <= prm.tol * bnorm:
            status = OK
            break
        cycles += 1
        tol_in = min(0.5, max(prm.tol * bnorm / rnorm, prm.tol_inner_floor))
        if method == "gmres":
            from .gmres import gmres_cycle
            if precond is not None or prm.replay is not None:
                raise ValueError("full-Arnoldi cycles take no preconditioner or rank replay")
            d, info = gmres_cycle(terms, r, Omega, prm, tol=tol_in, transpose=transpose, log=log)
        else:
            d, info = sgmres_cycle(terms, r, S, Omega, prm, tol=tol_in, transpose=transpose,
                                   log=log, replay=rep, precond=precond)
        iters += info["iters"]
        if x is None:
            x = d
        else:
            x, _ = roundsum([(1.0, x), (1.0, d)], Omega, rep.next(rpo))
        Rb = _residual_blocks(terms, B, x, transpose)
        rnorm = exact_norm(Rb)
        true_hist.append(rnorm / bnorm)
        if rnorm < best[0]:
            best = (rnorm, x)
        if rnorm <= prm.tol * bnorm:
            status = OK
            break
        h = true_hist[floor_from:]
        if len(h) >= 3 and h[-1] > 0.9 * h[-2] and h[-2] > 0.9 * h[-3]:
            if max(x.ranks) < prm.cap and rpo.eps > EPS_OUTER_MIN:
                rpo = dataclasses.replace(rpo, eps=max(1e-2 * rpo.eps, EPS_OUTER_MIN))
                floor_from = len(true_hist) - 1
            else:
                status = RANK_FLOOR
                break
        r, _ = roundsum(Rb, Omega, rep.next(rpo))
    if status != OK and best[1] is not None and best[0] < rnorm:
        rnorm, x = best
    if x is None:
        x = Tucker(np.zeros((1,) * B.d), [np.eye(nk, 1) for nk in B.n])
    return x, dict(status=status, iters=iters, cycles=cycles, true_hist=true_hist,
                   true_relres=rnorm / bnorm if bnorm > 0 else 0.0, seconds=time.perf_counter() - t0)
