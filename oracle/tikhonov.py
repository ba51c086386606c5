"""Projected Tikhonov regularisation of the sketched least squares, with the
regularisation parameter chosen by generalised cross validation (Sec. 4.3,
the projected problems for the deterministic and the sketched methods) --
oracle, test infrastructure only.

At iteration k the sketched methods minimise
    ||M_k y - b_s||^2 + lambda_k^2 ||y||^2,
M_k = [S vec L(V_1), ..., S vec L(V_k)] (s x k), b_s = S vec(B).

Definitions used here:
  * Reduction.  With the thin QR M_k = Q R (R k x k), c = Q^T b_s and
    rho = ||b_s - Q c||, the objective is ||R y - c||^2 + rho^2 +
    lambda^2 ||y||^2: the projected problem has k + 1 data, the coordinates
    of b_s in range(M_k) plus its orthogonal remainder, the same size as the
    Hessenberg problem of the deterministic method.
  * Solution.  With the SVD R = U diag(sigma) W^T and beta_hat = U^T c,
        y_lambda = W diag(sigma / (sigma^2 + lambda^2)) beta_hat,
        ||M_k y_lambda - b_s||^2
            = sum_i (lambda^2 / (sigma_i^2 + lambda^2))^2 beta_hat_i^2 + rho^2.
  * GCV (Golub, Heath and Wahba) on the projected problem (reading: the
    trace is taken over its k + 1 data, as in the hybrid projection methods
    the paper follows; over the s sketch rows the denominator would barely
    depend on lambda):
        G(lambda) = ||M_k y_lambda - b_s||^2 / trace(I_{k+1} - A_lambda)^2,
        trace(I_{k+1} - A_lambda) = 1 + sum_i lambda^2 / (sigma_i^2 + lambda^2),
    with A_lambda the influence matrix of the projected problem (a constant
    factor k + 1 in the numerator does not move the minimiser).
  * Minimiser (reading: the paper does not say how G is minimised).  G is
    evaluated on GCV_GRID points lambda_j = sigma_1 10^(-GCV_DECADES (1 - j /
    (GCV_GRID - 1))), the smallest value's index j* (first on ties) brackets
    a golden-section search in log10(lambda) over [lambda_{j*-1},
    lambda_{j*+1}] (clamped to the grid) with GCV_GOLDEN steps; the result is
    the bracket's midpoint unless the grid point is smaller.  lambda = 0 when
    M_k is zero.
"""
from __future__ import annotations

import numpy as np

GCV_GRID = 241          # 20 points per decade
GCV_DECADES = 12.0      # lambda / sigma_1 in [1e-12, 1]
GCV_GOLDEN = 60
_PHI = (np.sqrt(5.0) - 1.0) / 2.0


def reduce_ls(M: np.ndarray, b: np.ndarray):
    """Thin Householder QR of M: returns (R, c = Q^T b, rho = ||b - Q c||)."""
    Q, R = np.linalg.qr(M, mode="reduced")
    c = Q.T @ b
    rho = float(np.linalg.norm(b - Q @ c))
    return R, c, rho


def spectral_data(R: np.ndarray, c: np.ndarray):
    """SVD of R: singular values sigma, W (right vectors), beta_hat = U^T c."""
    U, sig, Wt = np.linalg.svd(R)
    return sig, Wt.T, U.T @ c


def _one_minus_filter(sig, lam):
    """1 - f = lambda^2 / (sigma^2 + lambda^2); where both vanish the filter
    factor f is 0 (the component is not fitted), so 1 - f = 1."""
    den = sig * sig + lam * lam
    return np.divide(lam * lam, den, out=np.ones_like(sig), where=den > 0)


def residual2(sig, bhat, rho, lam):
    """||M y_lambda - b_s||^2 through the filter factors."""
    g = _one_minus_filter(sig, lam)
    return float(np.sum((g * bhat) ** 2) + rho * rho)


def gcv(sig, bhat, rho, lam):
    """G(lambda) of the projected problem."""
    g = _one_minus_filter(sig, lam)
    return residual2(sig, bhat, rho, lam) / (1.0 + float(np.sum(g))) ** 2


def gcv_lambda(sig, bhat, rho) -> float:
    """Grid search, then golden-section refinement in log10(lambda)."""
    s1 = float(np.max(sig)) if len(sig) else 0.0
    if s1 == 0.0:
        return 0.0
    e = np.log10(s1) - GCV_DECADES * (1.0 - np.arange(GCV_GRID) / (GCV_GRID - 1))
    vals = np.array([gcv(sig, bhat, rho, 10.0 ** t) for t in e])
    j = int(np.argmin(vals))
    a, b = e[max(j - 1, 0)], e[min(j + 1, GCV_GRID - 1)]
    x1 = b - _PHI * (b - a)
    x2 = a + _PHI * (b - a)
    f1, f2 = gcv(sig, bhat, rho, 10.0 ** x1), gcv(sig, bhat, rho, 10.0 ** x2)
    for _ in range(GCV_GOLDEN):
        if f1 < f2:
            b, x2, f2 = x2, x1, f1
            x1 = b - _PHI * (b - a)
            f1 = gcv(sig, bhat, rho, 10.0 ** x1)
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + _PHI * (b - a)
            f2 = gcv(sig, bhat, rho, 10.0 ** x2)
    lam = 10.0 ** (0.5 * (a + b))
    return lam if gcv(sig, bhat, rho, lam) <= vals[j] else 10.0 ** e[j]


def tikhonov_solution(sig, W, bhat, lam):
    """y_lambda = W diag(sigma / (sigma^2 + lambda^2)) beta_hat (0 where
    sigma = lambda = 0)."""
    den = sig * sig + lam * lam
    f = np.divide(sig, den, out=np.zeros_like(sig), where=den > 0)
    return W @ (f * bhat)


def projected_tikhonov(M: np.ndarray, b: np.ndarray, lam=None):
    """Regularised sketched least squares.  ``lam`` None chooses lambda by GCV.
    Returns (y, ||M y - b||, lambda)."""
    R, c, rho = reduce_ls(M, b)
    sig, W, bhat = spectral_data(R, c)
    if lam is None:
        lam = gcv_lambda(sig, bhat, rho)
    y = tikhonov_solution(sig, W, bhat, lam)
    return y, float(np.sqrt(residual2(sig, bhat, rho, lam))), float(lam)
