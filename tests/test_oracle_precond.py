"""Pins of the exponential-sum inverse-Laplacian preconditioner and the
flexible sGMRES cycle (Sec. 3.4): closed forms, dense brute force on tiny
grids, and the dense solution."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from oracle import precond as P
from workloads import laplacian_1d


@pytest.mark.parametrize("n", [7, 16])
def test_dst1_diagonalises_the_1d_laplacian(n):
    V, lam = P.laplacian_eig(n)
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-14
    assert np.abs(V @ np.diag(lam) @ V.T - laplacian_1d(n)).max() <= 1e-13 * lam.max()
    assert np.allclose(np.sort(lam), np.linalg.eigvalsh(laplacian_1d(n)), rtol=1e-12)


@pytest.mark.parametrize("q,bound", [(16, 3.5e-2), (25, 1.5e-3), (36, 7e-5)])
def test_expsum_relative_error_over_the_poisson_spectrum(q, bound):
    # sum_h c_h exp(-t_h x) against 1/x on [3 lambda_1, 3 lambda_n] of the n = 32 grid;
    # the error falls with q (the sinc rule's step and range both improve)
    V, lam = P.laplacian_eig(32)
    x = np.geomspace(3 * lam[0], 3 * lam[-1], 4000)
    t, c = P.expsum(q)
    approx = (c[None, :] * np.exp(-np.outer(x, t))).sum(axis=1)
    assert np.max(np.abs(approx * x - 1)) <= bound


def test_spectral_application_equals_the_dense_exponential_sum():
    # M(X) through V_k^T U_k and row scalings equals the dense sum of Kronecker
    # products of matrix exponentials (scipy expm), and M inverts Delta_3 to the
    # exponential sum's accuracy
    rng = np.random.default_rng(0)
    n, q = 5, 25
    eig = [P.laplacian_eig(n)] * 3
    X = O.Tucker(rng.standard_normal((2, 3, 2)), [rng.standard_normal((n, r)) for r in (2, 3, 2)])
    t, c = P.expsum(q)
    L = laplacian_1d(n)
    Md = sum(ch * np.kron(np.kron(sl.expm(-th * L), sl.expm(-th * L)), sl.expm(-th * L)) for th, ch in zip(t, c))
    assert np.allclose(P.precond_dense(eig, q), Md, rtol=1e-10, atol=1e-14)
    MX = O.block_dense(P.expsum_blocks(X, eig, q))
    Xs = O.to_dense(X).ravel()
    V = eig[0][0]
    back = np.einsum("abc,ia,jb,kc->ijk", MX, V, V, V).ravel()
    assert np.linalg.norm(back - Md @ Xs) <= 1e-12 * np.linalg.norm(Md @ Xs)
    A = O.dense_operator([(1.0, [L if j == k else None for j in range(3)]) for k in range(3)], (n,) * 3)
    assert np.linalg.norm(Md @ A - np.eye(n ** 3), 2) <= 2e-3


def test_precond_apply_with_exact_rounding():
    # with a rounding that keeps everything (sketch covers the sum, eps = 0) the
    # rounded application equals the dense M applied to X
    rng = np.random.default_rng(1)
    n, q = 6, 16
    eig = [P.laplacian_eig(n)] * 3
    X = O.Tucker(rng.standard_normal((2, 2, 2)), [rng.standard_normal((n, 2)) for _ in range(3)])
    Om = [rng.standard_normal((n, n + 4)) for _ in range(3)]
    rp = O.RoundParams(eps=0.0, cap=n, p=4)
    Z = P.precond_apply(X, eig, q, lambda blocks: O.roundsum(blocks, Om, rp)[0])
    Md = P.precond_dense(eig, q)
    ref = Md @ O.to_dense(X).ravel()
    assert np.linalg.norm(O.to_dense(Z).ravel() - ref) <= 1e-10 * np.linalg.norm(ref)


def test_flexible_cycle_solves_poisson_in_few_iterations():
    # preconditioned flexible sGMRES on the n = 24 Poisson problem with the
    # separable right-hand side of the Laplacian experiment (ones/||ones|| x e_1 x e_1):
    # the true residual reaches 1e-8, far fewer iterations than without the
    # preconditioner, and the solution matches the dense solve
    n, q = 24, 36
    L = laplacian_1d(n)
    terms = [(1.0, [L if j == k else None for j in range(3)]) for k in range(3)]
    e1 = np.zeros((n, 1))
    e1[0] = 1.0
    B = O.Tucker(np.ones((1, 1, 1)), [np.ones((n, 1)) / np.sqrt(n), e1, e1])
    rng = np.random.default_rng(2)
    cap, p, s = 16, 5, 80
    S = [rng.standard_normal((n, s)) for _ in range(3)]
    Om = [rng.standard_normal((n, cap + p)) for _ in range(3)]
    eig = [P.laplacian_eig(n)] * 3
    prm = O.SGMRESParams(tol=1e-8, maxiter=40, k_trunc=2, cap=cap, p=p, max_restarts=6)
    Xp, ip = O.solve(terms, B, S, Om, prm, precond=lambda V, rf: P.precond_apply(V, eig, q, rf))
    assert ip["status"] == O.sgmres.OK and ip["true_relres"] <= 1e-8
    Xu, iu = O.solve(terms, B, S, Om, prm)
    assert ip["iters"] * 3 <= iu["iters"]
    A = O.dense_operator(terms, (n,) * 3)
    x = np.linalg.solve(A, O.to_dense(B).ravel())
    assert np.linalg.norm(O.to_dense(Xp).ravel() - x) <= 1e-6 * np.linalg.norm(x)
