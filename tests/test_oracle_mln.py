"""Pins of the MLN-Tucker sGMRES oracle (Sec. 3.3) against brute force on
tiny dense tensors, the paper's identities and special cases that reduce to
textbook computations."""
import numpy as np
import pytest

import oracle as O
from oracle import mln as M


def _rand_tucker(rng, n, r):
    return O.Tucker(rng.standard_normal(r), [rng.standard_normal((nk, rk)) for nk, rk in zip(n, r)])


def _kron_cols(mats, l):
    v = np.ones(1)
    for A in mats:
        v = np.kron(v, A[:, l])
    return v


def test_mln_sketch_against_dense():
    # G_Psi = X x_k Psi_k^T; F_k = X_(k) Omega_k with Omega_k the Khatri-Rao
    # product of the leading r columns of the other modes' Psi (row-major
    # unfolding order); diag(G_Psi) = (Psi_1 (.) ... (.) Psi_d)^T vec(X).
    rng = np.random.default_rng(0)
    n, r, p = (5, 6, 4), 3, 2
    blocks = [(0.7, _rand_tucker(rng, n, (2, 3, 2))), (-1.3, _rand_tucker(rng, n, (3, 1, 2)))]
    Psi = [rng.standard_normal((nk, r + p)) for nk in n]
    sk, diag = M.mln_sketch(blocks, Psi, r)
    X = O.block_dense(blocks)
    assert np.allclose(sk.core, O.multi_ttm(X, [P.T for P in Psi]), rtol=1e-12, atol=1e-12)
    for k in range(3):
        others = [Psi[j][:, :r] for j in range(3) if j != k]
        Om = np.stack([_kron_cols(others, l) for l in range(r)], axis=1)
        assert np.allclose(sk.F[k], O.unfold(X, k) @ Om, rtol=1e-12, atol=1e-10)
    dense_diag = np.array([_kron_cols(Psi, l) @ X.ravel() for l in range(r + p)])
    assert np.allclose(diag, dense_diag, rtol=1e-12, atol=1e-10)
    assert np.allclose(diag, O.sketch_krp(blocks, Psi), rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("ranks", [(2, 2, 2), (1, 1, 1)])
def test_mln_recovery_exact_below_the_target_rank(ranks):
    # Multilinear Nystrom is exact when every unfolding of the sum has rank
    # <= r; with rank < r, Psi_k^T F_k is rank deficient and R_k^+ is a true
    # pseudoinverse.
    rng = np.random.default_rng(1)
    n, r, p = (6, 5, 7), 5, 3
    blocks = [(1.0, _rand_tucker(rng, n, ranks)), (0.5, _rand_tucker(rng, n, ranks))]
    Psi = [rng.standard_normal((nk, r + p)) for nk in n]
    sk, _ = M.mln_sketch(blocks, Psi, r)
    Xt = M.mln_recovery(sk, Psi)
    X = O.block_dense(blocks)
    assert np.linalg.norm(O.to_dense(Xt) - X) <= 1e-10 * np.linalg.norm(X)


def test_mln_sum_is_the_sketch_of_the_sum():
    rng = np.random.default_rng(2)
    n, r, p = (5, 4, 6), 3, 2
    X1, X2 = _rand_tucker(rng, n, (2, 2, 3)), _rand_tucker(rng, n, (3, 2, 1))
    Psi = [rng.standard_normal((nk, r + p)) for nk in n]
    s1, _ = M.mln_sketch([(1.0, X1)], Psi, r)
    s2, _ = M.mln_sketch([(1.0, X2)], Psi, r)
    s12, _ = M.mln_sketch([(2.0, X1), (-0.5, X2)], Psi, r)
    s = M.mln_sum([s1, s2], [2.0, -0.5])
    assert np.allclose(s.core, s12.core, rtol=1e-12, atol=1e-12)
    for a, b in zip(s.F, s12.F):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def test_mln_memory_efficient_truncation_equals_smaller_sketch():
    # Keeping the leading r~_sol core indices and r_sol factor columns equals
    # sketching with the leading r~_sol columns of Psi_k and target r_sol.
    rng = np.random.default_rng(3)
    n, r, p, r_sol, p_sol = (7, 6, 5), 4, 4, 2, 2
    X = _rand_tucker(rng, n, (3, 4, 2))
    Psi = [rng.standard_normal((nk, r + p)) for nk in n]
    sk, _ = M.mln_sketch([(1.0, X)], Psi, r)
    t = M.truncate_sketch(sk, r_sol + p_sol, r_sol)
    ref, _ = M.mln_sketch([(1.0, X)], [P[:, :r_sol + p_sol] for P in Psi], r_sol)
    assert np.allclose(t.core, ref.core, rtol=1e-12, atol=1e-12)
    for a, b in zip(t.F, ref.F):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def _dense_sketched_gmres(A, b, S, maxiter, k_trunc, eta, tol):
    # The same short-recurrence sketched GMRES on vectors (classical
    # Gram-Schmidt over the window, sketched least squares).
    beta = np.linalg.norm(b)
    V = [b / beta]
    bs = S.T @ b
    cols, hist = [], []
    y = None
    for i in range(1, maxiter + 1):
        w = A @ V[-1]
        cols.append(S.T @ w)
        j0 = max(1, i - k_trunc + 1)
        h = [V[j - 1] @ w for j in range(j0, i + 1)]
        w = w - sum(hj * V[j - 1] for hj, j in zip(h, range(j0, i + 1)))
        Mm = np.stack(cols, axis=1)
        y, res, _ = O.sketched_lstsq(Mm, bs)
        hist.append(res / np.linalg.norm(bs))
        V.append(w / np.linalg.norm(w))
        if hist[-1] < eta * tol:
            break
    x = sum(yi * vi for yi, vi in zip(y, V))
    return x, hist


def test_mln_sgmres_reduces_to_dense_sketched_gmres():
    # With the target rank equal to the mode sizes the Nystrom recovery is
    # exact, and MLN-Tucker sGMRES is the vector sketched GMRES with the
    # Khatri-Rao sketch (Psi_1 (.) ... (.) Psi_d).
    rng = np.random.default_rng(4)
    n = 4
    from workloads import laplacian_1d
    L = laplacian_1d(n) / (n + 1) ** 2
    Dg = np.diag(rng.uniform(0.5, 1.5, n))
    terms = [(1.0, [L, None, None]), (1.0, [None, L, None]), (1.0, [None, None, L]), (0.3, [Dg, Dg, Dg])]
    B = _rand_tucker(rng, (n, n, n), (2, 1, 2))
    r, p = n, 16
    Psi = [rng.standard_normal((n, r + p)) for _ in range(3)]
    prm = M.MLNParams(r=r, p=p, tol=1e-10, maxiter=12, k_trunc=12)
    X, info = M.mln_sgmres(terms, B, Psi, prm)
    A = O.dense_operator(terms, (n, n, n))
    S = np.stack([_kron_cols(Psi, l) for l in range(r + p)], axis=1)
    x, hist = _dense_sketched_gmres(A, O.to_dense(B).ravel(), S, prm.maxiter, prm.k_trunc, prm.eta, prm.tol)
    assert len(hist) == len(info["hist"])
    assert np.allclose(info["hist"], hist, rtol=1e-8, atol=1e-13)
    assert np.linalg.norm(O.to_dense(X).ravel() - x) <= 1e-8 * np.linalg.norm(x)


def test_mln_sgmres_poisson_reaches_tolerance():
    # A tiny 3D Poisson problem with a full-rank target: the true residual of
    # the returned tensor reaches the tolerance and the solution matches the
    # dense solve.
    from workloads import laplacian_1d
    n = 6
    L = laplacian_1d(n)
    terms = [(1.0, [L if j == k else None for j in range(3)]) for k in range(3)]
    B = O.Tucker(np.ones((1, 1, 1)), [np.ones((n, 1))] * 3)
    rng = np.random.default_rng(5)
    r, p = n, 40
    Psi = [rng.standard_normal((n, r + p)) for _ in range(3)]
    X, info = M.mln_sgmres(terms, B, Psi, M.MLNParams(r=r, p=p, tol=1e-9, maxiter=40, k_trunc=40))
    assert info["status"] == O.sgmres.OK
    assert info["true_relres"] <= 1e-8
    A = O.dense_operator(terms, (n, n, n))
    x = np.linalg.solve(A, O.to_dense(B).ravel())
    assert np.linalg.norm(O.to_dense(X).ravel() - x) <= 1e-6 * np.linalg.norm(x)


def test_precond_blocks_equal_the_dense_exponential_sum():
    # The original-basis terms of M(X) that the flexible MLN method sketches
    # sum to the dense Kronecker exponential sum applied to vec(X).
    from oracle import precond as P
    rng = np.random.default_rng(6)
    n, q = 5, 16
    eig = [P.laplacian_eig(n)] * 3
    X = _rand_tucker(rng, (n, n, n), (2, 3, 2))
    got = O.block_dense(P.precond_blocks(X, eig, q)).ravel()
    ref = P.precond_dense(eig, q) @ O.to_dense(X).ravel()
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_flexible_mln_reduces_to_right_preconditioned_dense_gmres():
    # With the target rank equal to the mode sizes the Nystrom recovery is
    # exact, Z_k = M V_k, and the flexible MLN method is the vector sketched
    # GMRES on A M with the solution M (V y): same residual history, same
    # solution.  A wrong basis (sketching Z's spectral image) or the stored
    # V sketches in place of Z's would change the solution.
    from oracle import precond as P
    from workloads import laplacian_1d
    rng = np.random.default_rng(7)
    n, q = 4, 16
    L = laplacian_1d(n)
    terms = [(1.0, [L, None, None]), (1.0, [None, L, None]), (1.0, [None, None, L])]
    eig = [P.laplacian_eig(n)] * 3
    B = _rand_tucker(rng, (n, n, n), (2, 1, 2))
    r, p = n, 16
    Psi = [rng.standard_normal((n, r + p)) for _ in range(3)]
    prm = M.MLNParams(r=r, p=p, tol=1e-10, maxiter=10, k_trunc=10)
    X, info = M.mln_sgmres(terms, B, Psi, prm, precond=lambda V: P.precond_blocks(V, eig, q))
    A = O.dense_operator(terms, (n, n, n))
    Md = P.precond_dense(eig, q)
    S = np.stack([_kron_cols(Psi, l) for l in range(r + p)], axis=1)
    u, hist = _dense_sketched_gmres(A @ Md, O.to_dense(B).ravel(), S, prm.maxiter, prm.k_trunc, prm.eta, prm.tol)
    assert len(hist) == len(info["hist"])
    assert np.allclose(info["hist"], hist, rtol=1e-8, atol=1e-13)
    x = Md @ u
    assert np.linalg.norm(O.to_dense(X).ravel() - x) <= 1e-8 * np.linalg.norm(x)


@pytest.mark.parametrize("save_memory", [False, True])
def test_flexible_mln_poisson_in_few_iterations(save_memory):
    # The Laplacian experiment's right-hand side (ones/||ones|| x e_1 x e_1) on
    # the n = 16 grid at a target rank below n: the preconditioned MLN solve
    # reaches 1e-8 in far fewer iterations than the plain one and matches
    # the dense solution.
    from oracle import precond as P
    from workloads import laplacian_1d
    n, q = 16, 36
    L = laplacian_1d(n)
    terms = [(1.0, [L if j == k else None for j in range(3)]) for k in range(3)]
    e1 = np.zeros((n, 1))
    e1[0] = 1.0
    B = O.Tucker(np.ones((1, 1, 1)), [np.ones((n, 1)) / np.sqrt(n), e1, e1])
    eig = [P.laplacian_eig(n)] * 3
    rng = np.random.default_rng(8)
    r, p = 12, 4
    Psi = [rng.standard_normal((n, r + p)) for _ in range(3)]
    # the memory-efficient variant keeps 10 + 4 sketch indices of each Z
    prm = M.MLNParams(r=r, p=p, tol=1e-8, maxiter=40, k_trunc=3, save_memory=save_memory,
                      r_sol=10 if save_memory else r, p_sol=p)
    Xp, ip = M.mln_sgmres(terms, B, Psi, prm, precond=lambda V: P.precond_blocks(V, eig, q))
    Xu, iu = M.mln_sgmres(terms, B, Psi, prm)
    assert ip["status"] == O.sgmres.OK and ip["true_relres"] <= 1e-7
    assert ip["iters"] * 3 <= iu["iters"]
    A = O.dense_operator(terms, (n,) * 3)
    x = np.linalg.solve(A, O.to_dense(B).ravel())
    assert np.linalg.norm(O.to_dense(Xp).ravel() - x) <= (1e-5 if save_memory else 1e-6) * np.linalg.norm(x)
    if save_memory:
        assert max(Xp.ranks) <= 10
