"""Exponential-sum inverse-Laplacian preconditioner for Kronecker-sum
operators (Sec. 3.4, Eq. (Lap) and the exponential sum that follows it) --
oracle, test infrastructure only.

The 1D operator is Delta_1 = (n+1)^2 tridiag(-1, 2, -1) (n x n).  Its
eigenvectors are the DST-I basis and its eigenvalues are known in closed form:
    V[j, i] = sqrt(2/(n+1)) sin((i+1)(j+1) pi / (n+1)),
    lambda_i = 4 (n+1)^2 sin^2((i+1) pi / (2 (n+1))).
The inverse of the d-dimensional Laplacian is approximated by
    M = sum_{h=-q..q} c_h exp(-t_h Delta_1) (x) ... (x) exp(-t_h Delta_1),
    t_h = exp(h eta),  c_h = eta t_h,  eta = pi / sqrt(q),
the trapezoidal rule in s = log t for 1/x = int_0^inf exp(-t x) dt (reading:
the exponent carries a minus sign; with a plus sign the terms grow without
bound).  Through the eigendecomposition,
    M(X) = sum_h c_h G x_k (V_k exp(-t_h Lambda_k) V_k^T U_k)
for a Tucker tensor X = G x_k U_k: the transform V_k^T U_k (a DST-I of the
factor columns) is shared by all 2q + 1 terms, each term only rescales its
rows.

Rounded application T(M(X)) (the preconditioner of the flexible method): the
2q + 1 terms, which share the core, are rounded by RoundSum in the spectral
basis, i.e. on the block sum sum_h c_h G x_k (exp(-t_h Lambda_k) V_k^T U_k),
and the factors of the result are mapped back by V_k (reading: the paper
leaves the basis of the truncation open; V_k is orthogonal, so the rounded
tensor is the same up to the sketch's draw).
"""
from __future__ import annotations

from typing import Callable, List, Sequence, Tuple

import numpy as np

from .tucker import Tucker


def laplacian_eig(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """DST-I eigenvectors (columns) and eigenvalues of (n+1)^2 tridiag(-1, 2, -1)."""
    i = np.arange(1, n + 1)
    V = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(i, i) * np.pi / (n + 1))
    lam = 4.0 * (n + 1) ** 2 * np.sin(i * np.pi / (2 * (n + 1))) ** 2
    return V, lam


def expsum(q: int) -> Tuple[np.ndarray, np.ndarray]:
    """Nodes t_h and weights c_h, h = -q..q."""
    eta = np.pi / np.sqrt(q)
    h = np.arange(-q, q + 1)
    t = np.exp(h * eta)
    return t, eta * t


def expsum_blocks(X: Tucker, eig: Sequence[Tuple[np.ndarray, np.ndarray]], q: int):
    """The 2q + 1 terms of M(X) in the spectral basis,
    c_h G x_k (exp(-t_h Lambda_k) V_k^T U_k), each written with row scalings
    exp(-t_h (lambda - lambda_min,k)) (largest entry 1) and the coefficient
    c_h exp(-t_h sum_k lambda_min,k): the same tensor, with block coefficients
    that bound the blocks' size (RoundSum weighs blocks by |coef| ||core||)."""
    t, c = expsum(q)
    Ut = [V.T @ U for (V, _), U in zip(eig, X.U)]
    lmin = [float(np.min(lam)) for _, lam in eig]
    return [(float(ch * np.exp(-th * sum(lmin))),
             Tucker(X.core, [np.exp(-th * (lam - lm))[:, None] * u for (_, lam), lm, u in zip(eig, lmin, Ut)]))
            for th, ch in zip(t, c)]


def precond_blocks(X: Tucker, eig, q: int):
    """The 2q + 1 terms of M(X) in the basis of X,
    c_h G x_k (V_k exp(-t_h Lambda_k) V_k^T U_k), with the coefficients of
    ``expsum_blocks``.  The flexible MLN method sketches these terms (Sec. 3.4):
    the sketch of Z_k is stored and summed with the same Psi as every other
    sketch, so it is taken of the tensor itself, not of its spectral-basis
    image."""
    return [(c, Tucker(T.core, [V @ U for (V, _), U in zip(eig, T.U)])) for c, T in expsum_blocks(X, eig, q)]


def precond_apply(X: Tucker, eig, q: int, round_fn: Callable[[list], Tucker]) -> Tucker:
    """T(M(X)): round the spectral-basis terms with ``round_fn`` (a RoundSum of a
    block list) and map the factors back with V_k."""
    Zt = round_fn(expsum_blocks(X, eig, q))
    return Tucker(Zt.core, [V @ U for (V, _), U in zip(eig, Zt.U)])


def precond_dense(eig, q: int) -> np.ndarray:
    """Dense M (row-major vec), for tiny grids: sum_h c_h kron_k V_k exp(-t_h Lambda_k) V_k^T."""
    t, c = expsum(q)
    N = int(np.prod([V.shape[0] for V, _ in eig]))
    M = np.zeros((N, N))
    for th, ch in zip(t, c):
        K = np.ones((1, 1))
        for V, lam in eig:
            K = np.kron(K, (V * np.exp(-th * lam)) @ V.T)
        M += ch * K
    return M
