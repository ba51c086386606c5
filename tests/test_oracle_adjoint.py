"""Pins of the oracle's adjoint gradients: the dense FP64 gradient on a tiny
grid and central finite differences (CPU only)."""
import numpy as np

import oracle as O
from workloads import laplacian_1d


def _theta_problem(n, theta, rng):
    L = laplacian_1d(n)
    terms = [(float(theta[k]), [L if j == k else None for j in range(3)]) for k in range(3)]
    B = O.Tucker(np.ones((1, 1, 1)), [np.ones((n, 1))] * 3)
    Xt = O.Tucker(rng.standard_normal((2, 2, 2)), [rng.standard_normal((n, 2)) for _ in range(3)])
    return terms, B, Xt


def test_adjoint_matches_dense_gradient():
    rng = np.random.default_rng(0)
    n = 6
    theta = np.array([0.7, 1.3, 1.9])
    terms, B, Xt = _theta_problem(n, theta, rng)
    # add a non-identity factor in every mode of one term so dA has all modes
    A2 = [np.eye(n) + 0.1 * rng.standard_normal((n, n)) for _ in range(3)]
    terms.append((0.5, A2))
    S = [rng.standard_normal((n, 80)) for _ in range(3)]
    Om = [rng.standard_normal((n, 11)) for _ in range(3)]
    prm = O.SGMRESParams(tol=1e-13, maxiter=40, k_trunc=2, cap=6, p=5)
    x, info = O.solve(terms, B, S, Om, prm)
    assert info["true_relres"] <= 1e-13
    loss, xbar = O.loss_and_cotangent(x, Xt)
    lam, dalpha, dA, _ = O.adjoint_gradients(terms, x, xbar, S, Om, prm)
    Ld = O.dense_operator(terms, (n, n, n))
    xd = np.linalg.solve(Ld, O.to_dense(B).ravel())
    lam_d = np.linalg.solve(Ld.T, xd - O.to_dense(Xt).ravel())
    assert np.linalg.norm(O.to_dense(lam).ravel() - lam_d) <= 1e-9 * np.linalg.norm(lam_d)
    for j, (a, As) in enumerate(terms):
        K = O.dense_operator([(1.0, As)], (n, n, n))
        g = -lam_d @ (K @ xd)
        assert np.isclose(dalpha[j], g, rtol=1e-8, atol=1e-12 * abs(g) + 1e-300)
    # dA of the all-modes term: -alpha lam_(k) (kron_{l!=k} A^(l)) x_(k)^T
    X3, L3 = xd.reshape(n, n, n), lam_d.reshape(n, n, n)
    for k in range(3):
        Z = X3
        for l in range(3):
            if l != k:
                Z = O.ttm(Z, A2[l], l)
        ref = -0.5 * O.unfold(L3, k) @ O.unfold(Z, k).T
        assert np.allclose(dA[3][k], ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())


def test_adjoint_matches_central_differences():
    rng = np.random.default_rng(1)
    n = 10
    theta = np.array([0.8, 1.4, 0.6])
    terms, B, Xt = _theta_problem(n, theta, rng)
    S = [rng.standard_normal((n, 80)) for _ in range(3)]
    Om = [rng.standard_normal((n, 15)) for _ in range(3)]
    prm = O.SGMRESParams(tol=1e-13, maxiter=40, k_trunc=2, cap=n, p=5)   # no rank cap: exact solves

    def loss_at(th):
        tt = [(float(th[k]), As) for k, (_, As) in enumerate(terms)]
        x, info = O.solve(tt, B, S, Om, prm)
        return O.loss_and_cotangent(x, Xt)[0], x

    loss, x = loss_at(theta)
    _, xbar = O.loss_and_cotangent(x, Xt)
    lam, dalpha, _, _ = O.adjoint_gradients(terms, x, xbar, S, Om, prm, want_dA=False)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (loss_at(theta + e)[0] - loss_at(theta - e)[0]) / (2 * h)
        assert abs(fd - dalpha[k]) <= 1e-5 * abs(dalpha[k])
