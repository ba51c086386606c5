"""The rank certificate that lets the device settle the effective-rank rule
of RoundSum (Sec. 3.1) without the Gram's spectrum, checked against the
oracle's rule on constructed block sums.

The rule only feeds s = min(max_k r~_k + p, cap + p), so it suffices to know
whether some r~_k reaches the cap.  For any n x cap matrix Q with orthonormal
columns the Courant-Fischer theorem gives lambda_cap(G) >= lambda_min(Q^T G Q)
for the rule's Gram G = sum_b w_b^2 U_b U_b^T (w_b = |c_b| ||G_b||_F).  The
device takes Q = the first cap columns of the range-finder basis and declares
r~ >= cap when H - theta I has a Cholesky factorisation, H = Q^T G Q formed as
sum_b P_b P_b^T with P_b = w_b Q^T U_b, and
    theta = (4 max(delta, tau^2) + 4 (n sqrt(cap) + R) u) tr(G)
(R: columns of the concatenation, u: unit roundoff of the form).  Then
lambda_cap exceeds delta lambda_1 (it survives the zero clamp) and
tau^2 sum(lambda) (it alone exceeds the tail threshold), with a margin of 4
that covers the eigenvalue rounding of any backward-stable solver.

The certificate below restates that test in numpy (test code, not part of
the oracle); each case checks it against ``oracle.effective_sketch_size``:
it must never pass where the rule gives r~ < cap, it must pass on the
high-rank sums that the solver produces, and at the threshold it is the
conservative side that fails."""
import numpy as np
import pytest

import oracle as O
from oracle.roundsum import DELTA_CLAMP, RoundParams, effective_sketch_size

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def certificate(blocks, Qs, cap, tau, delta=DELTA_CLAMP, u=U64):
    """Per mode: does the Cholesky test settle r~_k >= cap?"""
    w = [abs(c) * np.linalg.norm(X.core.ravel()) for c, X in blocks]
    out = []
    for k, Q in enumerate(Qs):
        Qc = Q[:, :cap]
        P = [wb * (Qc.T @ X.U[k]) for wb, (_, X) in zip(w, blocks)]
        H = sum(Pb @ Pb.T for Pb in P)
        tr = sum(wb * wb * np.sum(X.U[k] ** 2) for wb, (_, X) in zip(w, blocks))
        n = Q.shape[0]
        R = sum(X.U[k].shape[1] for _, X in blocks)
        theta = (4.0 * max(delta, tau * tau) + 4.0 * (n * np.sqrt(cap) + R) * u) * tr
        try:
            np.linalg.cholesky(H - theta * np.eye(cap))
            out.append(True)
        except np.linalg.LinAlgError:
            out.append(False)
    return out


def range_bases(blocks, cap, p, rng):
    """Orthonormal bases of the range sketches Y_k = X_(k) KRP(Omega) of the
    sum (dense: small sizes only)."""
    X = sum(c * O.to_dense(T) for c, T in blocks)
    d = X.ndim
    Om = [rng.standard_normal((nk, cap + p)) for nk in X.shape]
    Qs = []
    for k in range(d):
        Xk = np.moveaxis(X, k, 0).reshape(X.shape[k], -1)
        others = [Om[j] for j in range(d) if j != k]
        K = others[0]
        for M in others[1:]:
            K = np.einsum("ia,ja->ija", K, M).reshape(-1, cap + p)
        Qs.append(np.linalg.qr(Xk @ K)[0])
    return Qs


def _orth(rng, n, r):
    return np.linalg.qr(rng.standard_normal((n, r)))[0]


@pytest.mark.parametrize("u", [U64, U32])
def test_passes_on_operator_like_sums(u):
    # L(V) = lambda V + (M x M x M) V with V rank cap: factors [U, M U]
    rng = np.random.default_rng(5)
    n, cap, p = (30, 28, 26), 12, 4
    U = [_orth(rng, nk, cap) for nk in n]
    M = [np.diag(np.linspace(1.0, 1e-3, nk)) @ _orth(rng, nk, nk) for nk in n]
    core = rng.standard_normal((cap,) * 3)
    blocks = [(1e-3, O.Tucker(core, U)), (1.0, O.Tucker(core, [Mk @ Uk for Mk, Uk in zip(M, U)]))]
    s, rt = effective_sketch_size(blocks, RoundParams(eps=1e-10, cap=cap, p=p))
    cert = certificate(blocks, range_bases(blocks, cap, p, rng), cap, tau=1e-10, u=u)
    assert s == cap + p and min(rt) >= cap
    assert all(cert)


def test_passes_on_orthogonalisation_sums():
    # W - sum_j h_j V_j with k_trunc = 2: three rank-cap blocks
    rng = np.random.default_rng(6)
    n, cap, p = (24, 24, 24), 10, 5
    blocks = []
    for c in (1.0, -0.3, 0.05):
        blocks.append((c, O.Tucker(rng.standard_normal((cap,) * 3), [_orth(rng, nk, cap) for nk in n])))
    s, rt = effective_sketch_size(blocks, RoundParams(eps=1e-10, cap=cap, p=p))
    assert s == cap + p
    assert all(certificate(blocks, range_bases(blocks, cap, p, rng), cap, tau=1e-10))


def test_fails_where_the_rule_stays_below_the_cap():
    # factors confined to a dim-dimensional subspace: lambda_cap(G) is rounding
    rng = np.random.default_rng(7)
    n, cap, p, dim = (26, 26, 26), 12, 4, 9
    B = [_orth(rng, nk, dim) for nk in n]
    blocks = [(rng.uniform(0.5, 2.0), O.Tucker(rng.standard_normal((cap,) * 3),
                                               [Bk @ rng.standard_normal((dim, cap)) for Bk in B]))
              for _ in range(4)]
    s, rt = effective_sketch_size(blocks, RoundParams(eps=1e-10, cap=cap, p=p))
    assert rt == [dim] * 3 and s == dim + p
    assert not any(certificate(blocks, range_bases(blocks, cap, p, rng), cap, tau=1e-10))


@pytest.mark.parametrize("tau", [1e-10, 1e-4])
@pytest.mark.parametrize("side", [-1, 1])
def test_threshold_is_conservative(tau, side):
    # cap - 1 unit eigenvalues from block 1 and a cap-th eigenvalue w2^2 from a
    # second block orthogonal to it; Q = the exact eigenbasis, so H is diagonal
    # and the Cholesky test passes exactly when w2^2 > theta
    rng = np.random.default_rng(8)
    n, cap = (40, 40, 40), 12
    Us = [_orth(rng, nk, cap) for nk in n]
    U1 = [Uk[:, :cap - 1] for Uk in Us]
    u2 = [Uk[:, cap - 1:] for Uk in Us]
    core1 = np.zeros((cap - 1,) * 3)
    for i in range(cap - 1):
        core1[i, i, i] = 1.0
    core1 /= np.linalg.norm(core1)
    tr1 = float(cap - 1)                      # w1 = 1, ||U1||_F^2 = cap - 1
    R = (cap - 1) + 1
    f = 4.0 * max(DELTA_CLAMP, tau * tau) + 4.0 * (n[0] * np.sqrt(cap) + R) * U64
    # w2^2 = f tr(G) (1 + side 1e-3), tr(G) = tr1 + w2^2
    lam = f * tr1 * (1 + side * 1e-3) / (1 - f * (1 + side * 1e-3))
    blocks = [(1.0, O.Tucker(core1, U1)), (np.sqrt(lam), O.Tucker(np.ones((1, 1, 1)), u2))]
    cert = certificate(blocks, Us, cap, tau=tau)
    s, rt = effective_sketch_size(blocks, RoundParams(eps=1e-10, cap=cap, p=3, tau=tau))
    assert cert == [side > 0] * 3
    # w2^2 is about 4 max(delta, tau^2) tr(G) on both sides: the rule keeps the
    # cap-th eigenvalue, so just below theta the certificate declines a case
    # the rule would settle at the cap (the conservative side; the device then
    # computes the spectrum)
    assert rt == [cap] * 3 and s == cap + 3


def test_never_passes_below_the_clamp():
    # the cap-th eigenvalue under delta lambda_1: the rule drops it (r~ = cap - 1)
    rng = np.random.default_rng(9)
    n, cap = (30, 30, 30), 10
    Us = [_orth(rng, nk, cap) for nk in n]
    core1 = np.zeros((cap - 1,) * 3)
    for i in range(cap - 1):
        core1[i, i, i] = 1.0
    blocks = [(1.0, O.Tucker(core1 / np.linalg.norm(core1), [Uk[:, :cap - 1] for Uk in Us])),
              (np.sqrt(0.5 * DELTA_CLAMP), O.Tucker(np.ones((1, 1, 1)), [Uk[:, cap - 1:] for Uk in Us]))]
    s, rt = effective_sketch_size(blocks, RoundParams(eps=1e-10, cap=cap, p=3))
    assert rt == [cap - 1] * 3
    assert not any(certificate(blocks, Us, cap, tau=1e-10))
