"""Seeded input generators (no method arithmetic): the structure the
workloads promise, checked on small sizes (CPU only)."""
import numpy as np

import workloads as W


def test_hollow_bars_is_outer_minus_inner_boxes():
    # each bar: indicator of an outer box minus the indicator of a box inside
    # it; the phantom is their sum and takes the values 0 and 1 only where
    # bars do not overlap
    n, nb = 24, 2
    core, U = W.hollow_bars(n, nb, np.random.default_rng(0))
    X = np.einsum("abc,ia,jb,kc->ijk", core, U[0], U[1], U[2])
    ref = np.zeros((n, n, n))
    for b in range(nb):
        o = [U[k][:, 2 * b] for k in range(3)]
        i = [U[k][:, 2 * b + 1] for k in range(3)]
        # the inner interval lies inside the outer one in every mode
        for k in range(3):
            assert np.all(i[k] <= o[k]) and i[k].sum() < o[k].sum()
        ref += np.einsum("i,j,k->ijk", *o) - np.einsum("i,j,k->ijk", *i)
    assert np.array_equal(X, ref)
    assert core.shape == (2 * nb,) * 3 and np.count_nonzero(core) == 2 * nb


def test_noisy_blur_problem_noise_level():
    K, Y, (Xc, XU), _ = W.noisy_blur_problem(12, seed=5, noise=0.05)
    clean = np.einsum("abc,ia,jb,kc->ijk", Xc, K @ XU[0], K @ XU[1], K @ XU[2])
    rel = np.linalg.norm(Y - clean) / np.linalg.norm(clean)
    assert 0.04 < rel < 0.06
    assert np.allclose(K, K.T) and np.all(K >= 0)


def test_deblur_gcv_problem_compression(tmp_path, monkeypatch):
    # the data are the truncated HOSVD of the noisy blurred phantom: orthonormal
    # factors of the requested rank, and the compressed tensor is the
    # projection of the noisy data onto their span
    monkeypatch.setenv("TSGMRES_CACHE", str(tmp_path))
    K, (core, Q), (Xc, XU) = W.deblur_gcv_problem(n=20, rank_b=6, seed=1)
    assert core.shape == (6, 6, 6) and all(q.shape == (20, 6) for q in Q)
    for q in Q:
        assert np.abs(q.T @ q - np.eye(6)).max() <= 1e-12
    # the compressed data stay close to the blurred phantom (5% noise, most of
    # it outside the rank-6 span)
    clean = np.einsum("abc,ia,jb,kc->ijk", Xc, K @ XU[0], K @ XU[1], K @ XU[2])
    comp = np.einsum("abc,ia,jb,kc->ijk", core, Q[0], Q[1], Q[2])
    assert np.linalg.norm(comp - clean) / np.linalg.norm(clean) < 0.05
    # cached: the same arrays come back
    K2, (core2, Q2), _ = W.deblur_gcv_problem(n=20, rank_b=6, seed=1)
    assert np.array_equal(core, core2) and all(np.array_equal(a, b) for a, b in zip(Q, Q2))


def test_laplacian_eigenpairs_diagonalise_the_1d_laplacian():
    # the closed-form DST-I pairs handed to the GPU preconditioner: V^T V = I
    # and V diag(lambda) V^T = (n+1)^2 tridiag(-1, 2, -1)
    from workloads import laplacian_1d, laplacian_eigenpairs
    Vs, lams = laplacian_eigenpairs([7, 16])
    for V, lam, n in zip(Vs, lams, [7, 16]):
        assert np.allclose(V.T @ V, np.eye(n), atol=1e-13)
        L = laplacian_1d(n)
        assert np.linalg.norm(V @ np.diag(lam) @ V.T - L) <= 1e-12 * np.linalg.norm(L)
