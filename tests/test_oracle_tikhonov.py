"""Pins of projected Tikhonov with GCV (Sec. 4.3): the regularised solution
against the stacked least-squares problem, the filter-factor GCV against the
influence matrix written out, the closed-form minimiser of equal singular
values, a brute-force minimisation on a fine grid, the lambda -> 0 limit, and
the regularising effect on a noisy deblurring problem."""
import numpy as np
import pytest

import oracle as O
from oracle import tikhonov as T


def _graded(rng, s, k, cond):
    # s x k with singular values from 1 down to 1/cond
    U, _ = np.linalg.qr(rng.standard_normal((s, k)))
    V, _ = np.linalg.qr(rng.standard_normal((k, k)))
    return U @ np.diag(np.geomspace(1.0, 1.0 / cond, k)) @ V.T


@pytest.mark.parametrize("k,lam", [(1, 0.3), (6, 1e-3), (20, 1e-5)])
def test_solution_equals_the_stacked_least_squares(k, lam):
    # argmin ||M y - b||^2 + lam^2 ||y||^2 = lstsq of [M; lam I] y ~ [b; 0]
    rng = np.random.default_rng(k)
    s = 40
    M = _graded(rng, s, k, 1e6)
    b = rng.standard_normal(s)
    y, res, lo = T.projected_tikhonov(M, b, lam=lam)
    assert lo == lam
    ref = np.linalg.lstsq(np.vstack([M, lam * np.eye(k)]), np.concatenate([b, np.zeros(k)]), rcond=None)[0]
    assert np.linalg.norm(y - ref) <= 1e-10 * np.linalg.norm(ref)
    assert abs(res - np.linalg.norm(M @ y - b)) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("k", [1, 5, 17])
def test_gcv_equals_the_influence_matrix_definition(k):
    # the projected problem [R; 0] y ~ [c; rho] with its influence matrix
    # A_lam = P (P^T P + lam^2 I)^{-1} P^T written out (P = [R; 0]), formed
    # stably as Q_top Q_top^T from the QR of the stacked [P; lam I]:
    # G = ||(I - A_lam) d||^2 / trace(I - A_lam)^2, and the numerator is the
    # s-row residual ||M y_lam - b||^2
    rng = np.random.default_rng(10 + k)
    s = 30
    M = _graded(rng, s, k, 1e4)
    b = rng.standard_normal(s)
    R, c, rho = T.reduce_ls(M, b)
    sig, W, bhat = T.spectral_data(R, c)
    P = np.vstack([R, np.zeros((1, k))])
    dvec = np.concatenate([c, [rho]])
    for lam in (1e-5, 1e-3, 0.1, 2.0):
        Qs, _ = np.linalg.qr(np.vstack([P, lam * np.eye(k)]))
        A = Qs[: k + 1] @ Qs[: k + 1].T
        I = np.eye(k + 1)
        num = np.linalg.norm((I - A) @ dvec) ** 2
        G = num / np.trace(I - A) ** 2
        assert abs(T.gcv(sig, bhat, rho, lam) - G) <= 1e-10 * G
        y = np.linalg.lstsq(np.vstack([M, lam * np.eye(k)]), np.concatenate([b, np.zeros(k)]), rcond=None)[0]
        assert abs(np.linalg.norm(M @ y - b) ** 2 - num) <= 1e-10 * num


@pytest.mark.parametrize("k,sigma", [(4, 1.0), (12, 3.0)])
def test_equal_singular_values_closed_form_minimiser(k, sigma):
    # R = sigma * orthogonal: with f = lam^2/(sigma^2+lam^2),
    # G = (f^2 B + rho^2) / (1 + k f)^2 (B = ||c||^2) is minimal at
    # f = k rho^2 / B, i.e. lam^2 = sigma^2 f / (1 - f)
    rng = np.random.default_rng(k)
    s = 3 * k + 5
    Qm, _ = np.linalg.qr(rng.standard_normal((s, k)))
    V, _ = np.linalg.qr(rng.standard_normal((k, k)))
    M = sigma * Qm @ V.T
    c = rng.standard_normal(k)
    perp = rng.standard_normal(s)
    perp -= Qm @ (Qm.T @ perp)
    perp *= 0.1 * np.linalg.norm(c) / np.sqrt(k) / np.linalg.norm(perp)   # f = 0.01
    b = Qm @ c + perp
    _, _, lam = T.projected_tikhonov(M, b)
    f = k * np.linalg.norm(perp) ** 2 / np.linalg.norm(c) ** 2
    lam_ref = sigma * np.sqrt(f / (1 - f))
    assert abs(lam / lam_ref - 1) <= 1e-7


def test_search_reaches_the_fine_grid_minimum():
    # brute force: G at the chosen lambda is no larger than its minimum over
    # 20001 points across the whole range
    rng = np.random.default_rng(3)
    for k, cond in [(8, 1e3), (25, 1e8), (40, 1e11)]:
        M = _graded(rng, 80, k, cond)
        xs = np.linalg.lstsq(M, rng.standard_normal(80), rcond=None)[0]
        b = M @ (xs / np.linalg.norm(xs)) + 1e-3 * rng.standard_normal(80)
        R, c, rho = T.reduce_ls(M, b)
        sig, W, bhat = T.spectral_data(R, c)
        lam = T.gcv_lambda(sig, bhat, rho)
        fine = np.geomspace(sig[0] * 1e-12, sig[0], 20001)
        gmin = min(T.gcv(sig, bhat, rho, x) for x in fine)
        assert T.gcv(sig, bhat, rho, lam) <= gmin * (1 + 1e-9)


def test_consistent_well_conditioned_problem_reduces_to_least_squares():
    # b in range(M): G(0) = 0, the choice is the grid's smallest lambda and y
    # is the unregularised sketched least-squares solution
    rng = np.random.default_rng(4)
    M = _graded(rng, 50, 10, 10.0)
    b = M @ rng.standard_normal(10)
    y, res, lam = T.projected_tikhonov(M, b)
    y0, res0, _ = O.sketched_lstsq(M, b)
    assert lam <= 1e-11 * np.linalg.norm(M, 2)
    assert np.linalg.norm(y - y0) <= 1e-12 * np.linalg.norm(y0)
    assert res <= 1e-12 * np.linalg.norm(b)


def test_zero_matrix_gives_zero_solution():
    y, res, lam = T.projected_tikhonov(np.zeros((10, 3)), np.ones(10))
    assert lam == 0.0 and np.all(y == 0) and abs(res - np.sqrt(10)) <= 1e-14


def _noisy_blur_problem(n, seed, noise):
    from workloads import noisy_blur_problem
    K, Y, (Xc, XU), rng = noisy_blur_problem(n, seed, noise)
    # full-rank Tucker form of the noisy data (identity factors): no compression
    B = O.Tucker(Y, [np.eye(n) for _ in range(3)])
    return [(1.0, [K, K, K])], B, O.Tucker(Xc, XU), rng


def test_gcv_regularises_a_noisy_blur_cycle():
    # the blurring operator is severely ill conditioned: without regularisation
    # the iterate after many iterations amplifies the noise (semiconvergence:
    # relative error 0.89 at 10 iterations, 1.96 at 30); with GCV it stays
    # near its best value (0.92)
    n = 10
    terms, B, Xt, rng = _noisy_blur_problem(n, 5, 0.05)
    cap, p, s, it = 10, 5, 60, 30
    S = [rng.standard_normal((n, s)) for _ in range(3)]
    Om = [rng.standard_normal((n, cap + p)) for _ in range(3)]
    xt = O.to_dense(Xt)

    def rre(prm):
        X, info = O.sgmres_cycle(terms, B, S, Om, prm, tol=1e-14)
        return np.linalg.norm(O.to_dense(X) - xt) / np.linalg.norm(xt), info

    e_plain, _ = rre(O.SGMRESParams(maxiter=it, k_trunc=2, cap=cap, p=p))
    e_gcv, info = rre(O.SGMRESParams(maxiter=it, k_trunc=2, cap=cap, p=p, tikhonov=True))
    assert len(info["lam"]) == info["iters"] and all(l > 0 for l in info["lam"][2:])
    assert e_gcv < 0.5 * e_plain
    assert e_gcv < 1.0
