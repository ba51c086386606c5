"""RHOSVD-Tucker GMRES (Alg. 1): full Arnoldi in Tucker format with every
sum recompressed by RoundSum -- oracle, test infrastructure only.

One cycle (``gmres_cycle``), in the steps of Alg. 1:
  beta = ||B||, V_1 = B / beta;
  for k = 1..N_max:
      W = RoundSum(L(V_k))
      h_{j,k} = <V_j, W> for j = 1..k               (all previous basis tensors)
      W = RoundSum(W - sum_j h_{j,k} V_j)
      h_{k+1,k} = ||W||
      y_k = argmin ||beta e_1 - H_{1:k+1,1:k} y||   (projected Tikhonov with GCV
                                                    instead, when asked: Sec. 4.3)
      res_k = ||beta e_1 - H y_k|| / beta
      if h_{k+1,k} ~ 0: stop;  V_{k+1} = W / h_{k+1,k}
      if res_k < tol: stop
  X = RoundSum(sum_i y_i V_i)

Readings, shared with the sketched cycle: the coefficients of one step all
come from the same W (one RoundSum of 1 + k blocks); y_k is computed before
the breakdown test, so a lucky breakdown returns the exact projected
solution; breakdown when h_{k+1,k} <= 1e-14 ||RoundSum(L V_k)|| or the new
diagonal of the Hessenberg least-squares R factor is <= 1e-14 ||H||_F.  The
convergence test is res_k < tol (Alg. 1 has no sketch correction factor).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from .roundsum import RoundParams, roundsum
from .sgmres import BREAKDOWN, NOT_CONVERGED, OK, SGMRESParams, sketched_lstsq
from .tikhonov import projected_tikhonov
from .tucker import Tucker, apply_op, exact_norm, inner, scale


def hessenberg_lstsq(H: np.ndarray, beta: float):
    """argmin ||beta e_1 - H y|| for the (k+1) x k Hessenberg H (Householder
    QR); returns (y, residual norm, |R_kk|)."""
    e1 = np.zeros(H.shape[0])
    e1[0] = beta
    return sketched_lstsq(H, e1)


def gmres_cycle(terms, B: Tucker, Omega, prm: SGMRESParams, tol: Optional[float] = None,
                transpose: bool = False, log: Optional[list] = None):
    """One cycle of Alg. 1 on ``L(X) = B``; returns (X, info).  Uses
    ``prm.maxiter``, ``cap``, ``p``, the RoundSum tolerances and
    ``prm.tikhonov``; ``k_trunc`` and the sketch are not used."""
    tol = prm.tol if tol is None else tol
    eps = prm.eps_trunc if prm.eps_trunc is not None else max(1e-2 * tol, prm.eps_min)
    rp = RoundParams(eps=eps, cap=prm.cap, p=prm.p)
    beta = exact_norm([(1.0, B)])
    V = [scale(B, 1.0 / beta)]
    H = np.zeros((prm.maxiter + 1, prm.maxiter))
    hist, lams = [], []
    status = NOT_CONVERGED
    y = np.zeros(0)
    k = 0
    for k in range(1, prm.maxiter + 1):
        W, i1 = roundsum(apply_op(terms, V[-1], transpose=transpose), Omega, rp)
        h = [inner(Vj, W) for Vj in V]
        W2, i2 = roundsum([(1.0, W)] + [(-hj, Vj) for hj, Vj in zip(h, V)], Omega, rp)
        omega = float(np.linalg.norm(W2.core.ravel()))
        wnorm = float(np.linalg.norm(W.core.ravel()))
        H[:k, k - 1] = h
        H[k, k - 1] = omega
        Hk = H[:k + 1, :k]
        y, res, rkk = hessenberg_lstsq(Hk, beta)
        if prm.tikhonov:
            e1 = np.zeros(k + 1)
            e1[0] = beta
            y, res, lam = projected_tikhonov(Hk, e1)
            lams.append(lam)
        rel = res / beta
        hist.append(rel)
        if log is not None:
            log.append(dict(k=k, s1=i1["s"], r1=i1["ranks"], s2=i2["s"], r2=i2["ranks"], h=h, omega=omega,
                            res=rel))
        if omega <= prm.breakdown_tol * wnorm or rkk <= prm.breakdown_tol * np.linalg.norm(Hk):
            status = BREAKDOWN
            break
        V.append(scale(W2, 1.0 / omega))
        if rel < tol:
            status = OK
            break
    X, i3 = roundsum([(float(y[i]), V[i]) for i in range(len(y))], Omega, rp)
    if log is not None:
        log.append(dict(final=True, s=i3["s"], r=i3["ranks"]))
    return X, dict(status=status, iters=k, hist=hist, beta=beta, lam=lams, H=H[:k + 1, :k].copy())
