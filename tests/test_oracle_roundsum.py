"""Pins of the oracle's RoundSum (Sec. 3.1): exactness, energy identity,
error bound, orthonormality and agreement with a deterministic truncated
HOSVD of the dense sum (CPU only)."""
import numpy as np
import pytest

import oracle as O
from oracle.roundsum import _rank_from_tail


def _rand_tucker(rng, n, r, orth=False):
    U = [rng.standard_normal((nk, rk)) for nk, rk in zip(n, r)]
    if orth:
        U = [np.linalg.qr(u)[0] for u in U]
    return O.Tucker(rng.standard_normal(tuple(r)), U)


def _omega(rng, n, width):
    return [rng.standard_normal((nk, width)) for nk in n]


@pytest.mark.parametrize("n", [(9, 8, 10), (6, 5, 6, 5)])
def test_exact_when_sketch_covers_rank(n):
    rng = np.random.default_rng(1)
    d = len(n)
    r1, r2 = (2,) * d, (3,) * d
    blocks = [(1.3, _rand_tucker(rng, n, r1)), (-0.4, _rand_tucker(rng, n, r2))]
    prm = O.RoundParams(eps=1e-15, cap=max(n), p=5)
    Om = _omega(rng, n, prm.cap + prm.p)
    X, info = O.roundsum(blocks, Om, prm)
    ref = O.block_dense(blocks)
    assert info["s"] >= 5
    assert np.linalg.norm(O.to_dense(X) - ref) <= 1e-12 * np.linalg.norm(ref)
    assert list(X.ranks) == [5] * d
    for u in X.U:
        assert np.allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-14)


def test_error_bound_and_ranks_match_dense_hosvd():
    rng = np.random.default_rng(2)
    n = (10, 9, 8)
    # a sum with decaying mode spectra
    base = _rand_tucker(rng, n, (6, 6, 6), orth=True)
    core = base.core * np.einsum("i,j,k->ijk", *[10.0 ** -np.arange(6)] * 3)
    blocks = [(1.0, O.Tucker(core, base.U)), (0.5, O.Tucker(0.1 * core, base.U))]
    eps = 1e-4
    prm = O.RoundParams(eps=eps, cap=10, p=5)
    X, info = O.roundsum(blocks, _omega(rng, n, 15), prm)
    dense = O.block_dense(blocks)
    err = np.linalg.norm(O.to_dense(X) - dense)
    assert err <= eps * np.linalg.norm(dense) * (1 + 1e-6)
    # deterministic ST-HOSVD of the dense sum, same rule, same modes order
    core_d, Vs, ranks = O.st_hosvd(dense, eps, 10)
    assert list(X.ranks) == ranks
    Xd = O.multi_ttm(core_d, Vs)
    assert np.linalg.norm(O.to_dense(X) - Xd) <= 1e-10 * np.linalg.norm(dense)


def test_st_hosvd_sequential_energy_identity():
    rng = np.random.default_rng(3)
    C = rng.standard_normal((7, 6, 5)) * np.einsum("i,j,k->ijk", 2.0 ** -np.arange(7), 2.0 ** -np.arange(6), 2.0 ** -np.arange(5))
    total = np.sum(C * C)
    eps = 5e-2
    core, Vs, ranks = O.st_hosvd(C, eps, 10)
    # discarded energy, mode by mode, from the singular values of the sequential unfoldings
    disc, T = 0.0, C
    for k in range(3):
        sig = np.linalg.svd(O.unfold(T, k), compute_uv=False)
        disc += np.sum(sig[ranks[k]:] ** 2)
        assert np.sum(sig[ranks[k]:] ** 2) <= eps * eps * total / 3 * (1 + 1e-12)
        T = O.ttm(T, Vs[k].T, k)
    assert np.isclose(np.sum(core * core) + disc, total, rtol=1e-12)


def test_forced_ranks_and_width_are_honoured():
    rng = np.random.default_rng(4)
    n = (8, 8, 8)
    blocks = [(1.0, _rand_tucker(rng, n, (4, 4, 4))), (1.0, _rand_tucker(rng, n, (3, 3, 3)))]
    prm = O.RoundParams(eps=1e-12, cap=8, p=3, force_s=6, force_ranks=(2, 3, 4))
    X, info = O.roundsum(blocks, _omega(rng, n, 11), prm)
    assert info["s"] == 6 and list(X.ranks) == [2, 3, 4]


def test_effective_rank_invariances():
    rng = np.random.default_rng(5)
    n = (12, 11, 10)
    X, Y = _rand_tucker(rng, n, (3, 2, 3)), _rand_tucker(rng, n, (2, 3, 1))
    prm = O.RoundParams(eps=1e-10, cap=20, p=5)
    s1, rt1 = O.effective_sketch_size([(1.0, X), (2.0, Y)], prm)
    # splitting a summand into two equal halves leaves the estimate unchanged
    s2, rt2 = O.effective_sketch_size([(0.5, X), (0.5, X), (2.0, Y)], prm)
    # a global scale leaves it unchanged too
    s3, rt3 = O.effective_sketch_size([(1e3, X), (2e3, Y)], prm)
    assert rt1 == rt2 == rt3 and s1 == s2 == s3
    assert rt1 == [5, 5, 4]          # generic ranks of the concatenations
    # the width is capped at cap + p, while the per-mode estimates stay exact
    prm2 = O.RoundParams(eps=1e-10, cap=4, p=2)
    s4, rt4 = O.effective_sketch_size([(1.0, X), (2.0, Y)], prm2)
    assert rt4 == [5, 5, 4] and s4 == 6


def _orthonormal_blocks(rng, n, ranks):
    """Factors whose columns are orthonormal ACROSS the blocks, so that the
    weighted Gram sum_b w_b^2 U_b U_b^T has the eigenvalues w_b^2 with
    multiplicity r_b exactly (in every mode)."""
    d = len(n)
    tot = sum(r for r in ranks)
    Q = [np.linalg.qr(rng.standard_normal((nk, tot)))[0] for nk in n]
    out, off = [], 0
    for r in ranks:
        out.append([Q[k][:, off:off + r] for k in range(d)])
        off += r
    return out


@pytest.mark.parametrize("side", ["below", "above"])
def test_effective_rank_threshold_is_exact(side):
    """Pin of the Sec. 3.1 rule's threshold and weighting.  Block 1: c = 1,
    ||G|| = 1, rank 2 -> Gram eigenvalue 1 (twice).  Block 2: c = 1e-3,
    ||G|| = 2, rank 1 -> eigenvalue (|c| ||G||)^2 = 4e-6.  The tail beyond
    r = 2 is exactly 4e-6, so tau^2 sum(lambda) just below it gives r~ = 3 and
    just above gives r~ = 2.  Weights |c| (no core norm: tail 1e-6), |c| ||G||^2
    (tail 1.6e-5), ||G|| (tail 4) or an unsquared Gram (tail 2e-3) each flip
    one of the two cases."""
    rng = np.random.default_rng(11)
    n = (9, 8, 7)
    f1, f2 = _orthonormal_blocks(rng, n, [2, 1])
    G1 = rng.standard_normal((2, 2, 2))
    G1 /= np.linalg.norm(G1)
    G2 = np.full((1, 1, 1), 2.0)
    blocks = [(1.0, O.Tucker(G1, f1)), (-1e-3, O.Tucker(G2, f2))]
    total = 2.0 + 4e-6
    thr = 4e-6 * (1.0 - 1e-6 if side == "below" else 1.0 + 1e-6)
    prm = O.RoundParams(eps=1e-10, cap=8, p=2, tau=np.sqrt(thr / total))
    s, rt = O.effective_sketch_size(blocks, prm)
    want = 3 if side == "below" else 2
    assert rt == [want] * 3 and s == want + 2


def test_effective_rank_wide_concatenation_is_numerical_rank():
    """Past every kernel-size boundary (n = 200 and R = 240 columns) the rule
    runs on the n-side Gram: with a tiny tau it returns the numerical rank of
    the weighted concatenation, counted here independently from its SVD."""
    rng = np.random.default_rng(12)
    n = (200, 170, 190)
    B = [np.linalg.qr(rng.standard_normal((nk, 100)))[0] for nk in n]   # 100-dim subspaces
    blocks = []
    for b in range(30):
        U = [Bk @ rng.standard_normal((100, 8)) for Bk in B]
        blocks.append((float(rng.uniform(0.5, 2.0)), O.Tucker(rng.standard_normal((8, 8, 8)), U)))
    prm = O.RoundParams(eps=1e-13, cap=120, p=5)
    s, rt = O.effective_sketch_size(blocks, prm)
    for k in range(3):
        V = np.concatenate([abs(c) * np.linalg.norm(X.core) * X.U[k] for c, X in blocks], axis=1)
        sv = np.linalg.svd(V, compute_uv=False)
        assert rt[k] == int(np.sum(sv > 1e-5 * sv[0])) == 100
    assert s == 105


def test_rank_tail_rule():
    v = np.array([4.0, 1.0, 0.25, 0.0])
    assert _rank_from_tail(v, 0.25) == 2
    assert _rank_from_tail(v, 0.2) == 3
    assert _rank_from_tail(v, 0.0) == 3
    assert _rank_from_tail(v, 10.0) == 0


def test_zero_sum_returns_rank_one_zero():
    rng = np.random.default_rng(6)
    n = (5, 5, 5)
    X = _rand_tucker(rng, n, (2, 2, 2))
    Z, info = O.roundsum([(1.0, X), (-1.0, X)], _omega(rng, n, 8), O.RoundParams(eps=1e-10, cap=4, p=2))
    assert Z.ranks == (1, 1, 1) and np.all(Z.core == 0)
