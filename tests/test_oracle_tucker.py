"""Pins of the oracle's Tucker primitives against brute force and closed
forms (CPU only)."""
import numpy as np
import pytest

import oracle as O


def _rand_tucker(rng, n, r):
    return O.Tucker(rng.standard_normal(tuple(r)), [rng.standard_normal((nk, rk)) for nk, rk in zip(n, r)])


def _rand_terms(rng, n, nterms=3, ident_prob=0.4):
    terms = []
    for j in range(nterms):
        As = [None if rng.random() < ident_prob else rng.standard_normal((nk, nk)) for nk in n]
        terms.append((float(rng.uniform(0.5, 2.0)), As))
    return terms


@pytest.mark.parametrize("n,r", [((5, 4, 6), (2, 3, 2)), ((4, 3, 4, 3), (2, 2, 3, 1))])
@pytest.mark.parametrize("transpose", [False, True])
def test_apply_matches_dense_kronecker(n, r, transpose):
    rng = np.random.default_rng(11)
    X = _rand_tucker(rng, n, r)
    terms = _rand_terms(rng, n)
    Ld = O.dense_operator(terms, n)
    if transpose:
        Ld = Ld.T
    ref = Ld @ O.to_dense(X).ravel()
    got = O.block_dense(O.apply_op(terms, X, transpose=transpose)).ravel()
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-12 * np.abs(ref).max())


def test_poisson_sine_eigentensor():
    # L v_j = lambda_j v_j with lambda_j = 4 (n+1)^2 sin^2(j pi / (2(n+1)))  (Sec. 3.4, DST-I)
    n = 9
    from workloads import laplacian_1d
    L = laplacian_1d(n)
    idx = np.arange(1, n + 1)
    js = (2, 5, 7)
    v = [np.sin(idx * j * np.pi / (n + 1))[:, None] for j in js]
    lam = [4 * (n + 1) ** 2 * np.sin(j * np.pi / (2 * (n + 1))) ** 2 for j in js]
    X = O.Tucker(np.ones((1, 1, 1)), v)
    terms = [(1.0, [L if a == k else None for a in range(3)]) for k in range(3)]
    got = O.block_dense(O.apply_op(terms, X))
    assert np.allclose(got, sum(lam) * O.to_dense(X), rtol=1e-12, atol=1e-9)


def _krp(mats):
    s = mats[0].shape[1]
    cols = []
    for l in range(s):
        c = np.ones(1)
        for M in mats:
            c = np.kron(c, M[:, l])
        cols.append(c)
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("n,r,s", [((5, 4, 6), (2, 3, 2), 7), ((3, 4, 3, 2), (2, 2, 1, 2), 5)])
def test_sketch_matches_dense_khatri_rao(n, r, s):
    rng = np.random.default_rng(5)
    blocks = [(1.5, _rand_tucker(rng, n, r)), (-0.25, _rand_tucker(rng, n, r[::-1] if len(set(n)) == 1 else r))]
    S = [rng.standard_normal((nk, s)) for nk in n]
    ref = _krp(S).T @ O.block_dense(blocks).ravel()
    got = O.sketch_krp(blocks, S)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_sketch_superdiagonal_identity():
    # diag(X x_k S_k^T) = (S_1 (.) ... (.) S_d)^T vec(X)   (Sec. 3.3)
    rng = np.random.default_rng(6)
    n, r, s = (6, 5, 4), (3, 2, 2), 4
    blocks = [(1.0, _rand_tucker(rng, n, r)), (0.5, _rand_tucker(rng, n, r))]
    S = [rng.standard_normal((nk, s)) for nk in n]
    full = O.sketch_kron(blocks, S)
    diag = np.array([full[l, l, l] for l in range(s)])
    assert np.allclose(diag, O.sketch_krp(blocks, S), rtol=1e-12)


def test_sketch_linear_over_blocks():
    rng = np.random.default_rng(7)
    n, r, s = (7, 6, 5), (2, 3, 2), 9
    X, Y = _rand_tucker(rng, n, r), _rand_tucker(rng, n, r)
    S = [rng.standard_normal((nk, s)) for nk in n]
    lhs = O.sketch_krp([(2.0, X), (-3.0, Y)], S)
    rhs = 2.0 * O.sketch_krp([(1.0, X)], S) - 3.0 * O.sketch_krp([(1.0, Y)], S)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())


def test_inner_and_norm_match_dense():
    rng = np.random.default_rng(8)
    n = (6, 5, 7)
    X, Y = _rand_tucker(rng, n, (2, 3, 2)), _rand_tucker(rng, n, (3, 2, 4))
    assert np.isclose(O.inner(X, Y), np.sum(O.to_dense(X) * O.to_dense(Y)), rtol=1e-12)
    blocks = [(1.0, X), (-0.7, Y), (0.2, X)]
    assert np.isclose(O.exact_norm(blocks), np.linalg.norm(O.block_dense(blocks)), rtol=1e-12)


def test_exact_norm_no_cancellation():
    # ||(B + delta E) - B|| with delta ||E|| / ||B|| = 1e-12 is recovered to 1%,
    # though the two terms agree to 12 digits.
    rng = np.random.default_rng(9)
    n = (12, 10, 11)
    B = _rand_tucker(rng, n, (3, 3, 3))
    E = _rand_tucker(rng, n, (2, 2, 2))
    nb, ne = np.linalg.norm(O.to_dense(B)), np.linalg.norm(O.to_dense(E))
    delta = 1e-12 * nb / ne
    # B2 = B + delta E as one Tucker tensor with concatenated factors
    core = np.zeros((5, 5, 5))
    core[:3, :3, :3] = B.core
    core[3:, 3:, 3:] = delta * E.core
    B2 = O.Tucker(core, [np.concatenate([u, v], axis=1) for u, v in zip(B.U, E.U)])
    got = O.exact_norm([(1.0, B2), (-1.0, B)])
    assert abs(got / (delta * ne) - 1.0) < 1e-2


def test_storage_worked_example():
    # Worked example printed in the paper (fixture carries the citation):
    # Tucker storage sum_k n_k r_k + prod_k r_k of the deblurring right-hand side.
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "storage_example.json")))
    n, r = g["n"], g["ranks"]
    assert sum(a * b for a, b in zip(n, r)) + int(np.prod(r)) == g["tucker_floats"]
    assert int(np.prod(n)) == g["dense_floats"]
