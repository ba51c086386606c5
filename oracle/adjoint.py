"""Adjoint of the Tucker sGMRES solve -- oracle, test infrastructure only.

For ``L(x) = b`` with ``L = sum_j alpha_j A_j^(1) kron ... kron A_j^(d)``
(Eq. (2)) and a loss l(x) with cotangent x_bar = dl/dx:
  * lambda solves ``L^T lambda = x_bar`` (the same restarted Tucker sGMRES on
    the transposed factors);
  * dl/db = lambda;
  * dl/dalpha_j = -<lambda, x x_1 A_j^(1) ... x_d A_j^(d)>;
  * dl/dA_j^(k) = -alpha_j lambda_(k) (kron_{l!=k} A_j^(l)) x_(k)^T, which in
    Tucker form is ``-alpha_j U^lam_k Mid U^x_k^T`` with
    ``Mid = G^lam_(k) (kron_{l!=k} P_l) G^x_(k)^T``,
    ``P_l = U^lam_l^T A_j^(l) U^x_l`` (identity factors give U^lam^T U^x).
The gradient formulas follow by differentiating Eq. (2); the paper itself
has no adjoint.
"""
from __future__ import annotations

import numpy as np

from .roundsum import RoundParams, roundsum
from .sgmres import SGMRESParams, solve
from .tucker import Tucker, exact_norm, inner, multi_ttm, transpose_terms, unfold


def loss_and_cotangent(x: Tucker, x_target: Tucker):
    """l = ||x - x_t||^2 / 2 (exact norm) and its cotangent x_bar = x - x_t
    as a two-block sum."""
    blocks = [(1.0, x), (-1.0, x_target)]
    return 0.5 * exact_norm(blocks) ** 2, blocks


def _term_tensor(x: Tucker, As):
    """x x_1 A^(1) ... x_d A^(d) as a Tucker tensor (shared core)."""
    return Tucker(x.core, [u if A is None else A @ u for A, u in zip(As, x.U)])


def adjoint_gradients(terms, x: Tucker, xbar_blocks, S, Omega, prm: SGMRESParams,
                      want_dA: bool = True):
    """Returns (lambda, dalpha[nterms], dA[j][k] or None)."""
    eps = 1e-2 * prm.tol
    xb, _ = roundsum(xbar_blocks, Omega, RoundParams(eps=eps, cap=prm.cap, p=prm.p))
    lam, info = solve(transpose_terms(terms), xb, S, Omega, prm)
    dalpha = np.array([-inner(lam, _term_tensor(x, As)) for _, As in terms])
    dA = None
    if want_dA:
        dA = []
        d = x.d
        for a, As in terms:
            row = []
            for k in range(d):
                if As[k] is None:
                    row.append(None)
                    continue
                P = [lam.U[l].T @ (x.U[l] if As[l] is None else As[l] @ x.U[l]) for l in range(d)]
                H = multi_ttm(x.core, [None if l == k else P[l] for l in range(d)])
                Mid = unfold(lam.core, k) @ unfold(H, k).T
                row.append(-a * lam.U[k] @ Mid @ x.U[k].T)
            dA.append(row)
    return lam, dalpha, dA, info
