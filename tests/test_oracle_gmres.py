"""Pins of the oracle's RHOSVD-Tucker GMRES (Alg. 1, full Arnoldi): dense
textbook GMRES when the RoundSums are exact, the Arnoldi relation and the
orthonormality of the basis, the Poisson closed form, lucky breakdown on an
eigentensor, and the Hessenberg form of projected Tikhonov (CPU only)."""
import numpy as np
import pytest

import oracle as O
from oracle.gmres import gmres_cycle
from oracle.sgmres import BREAKDOWN, OK
from workloads import laplacian_1d, make_config
from test_oracle_sgmres import _poisson_exact, _random_problem, _textbook_gmres_history


def test_textbook_gmres_reduction():
    # exact RoundSums (cap >= n, eps 1e-15): the residual history is dense GMRES
    rng = np.random.default_rng(0)
    n = (4, 3, 4)
    terms, B = _random_problem(rng, n)
    Om = [rng.standard_normal((nk, max(n) + 5)) for nk in n]
    kmax = 14
    prm = O.SGMRESParams(maxiter=kmax, cap=max(n), p=5, eps_trunc=1e-15)
    X, info = gmres_cycle(terms, B, Om, prm, tol=1e-30)
    ref = _textbook_gmres_history(O.dense_operator(terms, n), O.to_dense(B).ravel(), kmax)
    assert len(info["hist"]) == kmax
    assert np.allclose(info["hist"], ref, rtol=1e-8, atol=1e-13)


def test_arnoldi_relation_and_orthonormal_basis():
    # L(V_k) = sum_{j <= k+1} H[j, k] V_j (dense rebuild from the logged
    # coefficients) and <V_i, V_j> = delta_ij
    rng = np.random.default_rng(1)
    n = (5, 4, 5)
    terms, B = _random_problem(rng, n)
    Om = [rng.standard_normal((nk, 10)) for nk in n]
    prm = O.SGMRESParams(maxiter=8, cap=5, p=5, eps_trunc=1e-15)
    log = []
    X, info = gmres_cycle(terms, B, Om, prm, tol=1e-30, log=log)
    Ld = O.dense_operator(terms, n)
    b = O.to_dense(B).ravel()
    V = [b / np.linalg.norm(b)]
    H = info["H"]
    for entry in log[:-1]:
        k = entry["k"]
        w = Ld @ V[-1]
        w2 = w - sum(h * v for h, v in zip(entry["h"], V))
        assert np.isclose(np.linalg.norm(w2), H[k, k - 1], rtol=1e-9)
        V.append(w2 / H[k, k - 1])
    Vm = np.stack(V, axis=1)
    assert np.abs(Vm.T @ Vm - np.eye(Vm.shape[1])).max() <= 1e-10
    kk = H.shape[1]
    assert np.linalg.norm(Ld @ Vm[:, :kk] - Vm[:, :kk + 1] @ H) <= 1e-10 * np.linalg.norm(Ld @ Vm[:, :kk])
    # the returned solution is sum y_i V_i with y the Hessenberg least squares
    e1 = np.zeros(kk + 1)
    e1[0] = np.linalg.norm(b)
    y = np.linalg.lstsq(H, e1, rcond=None)[0]
    assert np.linalg.norm(O.to_dense(X).ravel() - Vm[:, :kk] @ y) <= 1e-10 * np.linalg.norm(Vm[:, :kk] @ y)


def test_restarted_full_arnoldi_solves_poisson():
    w = make_config(1, n=12, cap=12)
    B = O.Tucker(w.b_core, w.b_factors)
    prm = O.SGMRESParams(tol=1e-10, maxiter=40, cap=12, p=w.p)
    X, info = O.solve(w.terms, B, None, w.Omega, prm, method="gmres")
    assert info["status"] == OK and info["true_relres"] <= 1e-10
    Xe = _poisson_exact(12, B)
    assert np.linalg.norm(O.to_dense(X) - Xe) <= 1e-7 * np.linalg.norm(Xe)


def test_full_arnoldi_needs_no_more_iterations_than_truncated():
    # on the same problem, the full-Arnoldi cycle (exact minimal residual over
    # the Krylov space) needs at most as many iterations as the truncated,
    # sketched one to reach the same sketched/true tolerance
    rng = np.random.default_rng(3)
    n = (6, 5, 6)
    terms, B = _random_problem(rng, n)
    S = [rng.standard_normal((nk, 60)) for nk in n]
    Om = [rng.standard_normal((nk, 11)) for nk in n]
    prm = O.SGMRESParams(maxiter=30, k_trunc=2, cap=6, p=5)
    _, ig = gmres_cycle(terms, B, Om, prm, tol=1e-8)
    _, isg = O.sgmres_cycle(terms, B, S, Om, prm, tol=1e-8)
    assert ig["status"] == OK and ig["iters"] <= isg["iters"]


def test_lucky_breakdown_on_eigentensor():
    n = 12
    L = laplacian_1d(n)
    idx = np.arange(1, n + 1)
    v = [np.sin(idx * j * np.pi / (n + 1))[:, None] for j in (1, 2, 3)]
    B = O.Tucker(np.ones((1, 1, 1)), v)
    terms = [(1.0, [L if a == k else None for a in range(3)]) for k in range(3)]
    Om = [np.random.default_rng(4).standard_normal((n, 9)) for _ in range(3)]
    X, info = gmres_cycle(terms, B, Om, O.SGMRESParams(maxiter=10, cap=4, p=5), tol=1e-12)
    assert info["status"] == BREAKDOWN and info["iters"] == 1
    lam = sum(4 * (n + 1) ** 2 * np.sin(j * np.pi / (2 * (n + 1))) ** 2 for j in (1, 2, 3))
    assert np.allclose(O.to_dense(X), O.to_dense(B) / lam, rtol=1e-10, atol=1e-14)


def test_hessenberg_tikhonov_regularises_noisy_blur():
    # projected Tikhonov on the Hessenberg problem (Sec. 4.3): after 30
    # full-Arnoldi iterations the unregularised reconstruction error is 5.6
    # (noise amplified), the regularised one 0.92
    from workloads import noisy_blur_problem
    n = 10
    K, Y, (Xc, XU), rng = noisy_blur_problem(n, 5, 0.05)
    terms = [(1.0, [K, K, K])]
    B = O.Tucker(Y, [np.eye(n) for _ in range(3)])
    Om = [rng.standard_normal((n, n + 5)) for _ in range(3)]
    xt = O.to_dense(O.Tucker(Xc, XU))
    errs = []
    for tik in (False, True):
        X, info = gmres_cycle(terms, B, Om, O.SGMRESParams(maxiter=30, cap=n, p=5, tikhonov=tik), tol=1e-14)
        errs.append(np.linalg.norm(O.to_dense(X) - xt) / np.linalg.norm(xt))
    assert errs[1] < 0.5 * errs[0] and errs[1] < 1.0
