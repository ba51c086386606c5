"""The one-count shortcut of the effective-rank rule (Sec. 3.1) that the
device's eigenvalue kernels take when the caller only needs min(r~, cap):
one Sturm count tells whether at least cap eigenvalues of the rule's Gram lie
at or above

    x = max(tau^2 tot, delta (gu + t)) + 2 t,
    tot = trace + N (max(0, -gl) + t),

with gl <= lambda_min <= lambda_max <= gu (Gershgorin bounds) and t the
multisection tolerance 2 u max(|gl|, |gu|).  If so, the cap-th largest
eigenvalue survives the delta clamp and alone exceeds tau^2 times the rule's
total, so r~ >= cap and the multisection is skipped.

The test restates that condition in numpy (test code, not part of the
oracle) with the tightest admissible bounds (gl = lambda_min, gu =
lambda_max, an exact count), which makes it the least conservative version,
and checks it against ``oracle.effective_sketch_size``: it must never hold
where the rule gives r~ < cap, and it must hold on the high-rank sums that
the solver produces."""
import numpy as np
import pytest

import oracle as O
from oracle.roundsum import DELTA_CLAMP, RoundParams, effective_sketch_size

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def shortcut(blocks, cap, tau, delta=DELTA_CLAMP, u=U64):
    """Per mode: does the one-count test settle r~_k >= cap?"""
    w = [abs(c) * np.linalg.norm(X.core.ravel()) for c, X in blocks]
    out = []
    for k in range(blocks[0][1].d):
        V = np.concatenate([wb * X.U[k] for wb, (_, X) in zip(w, blocks)], axis=1)
        G = V.T @ V if V.shape[1] <= V.shape[0] else V @ V.T
        lam = np.linalg.eigvalsh(G)
        N = lam.size
        if cap > N:
            out.append(False)
            continue
        gl, gu = lam[0], lam[-1]
        t = 2.0 * u * max(abs(gl), abs(gu))
        tot = np.trace(G) + N * (max(0.0, -gl) + t)
        x = max(tau * tau * tot, delta * (gu + t)) + 2.0 * t
        out.append(int(np.sum(lam >= x)) >= cap)
    return out


def _orth(rng, n, r):
    return np.linalg.qr(rng.standard_normal((n, r)))[0]


@pytest.mark.parametrize("u", [U64, U32])
def test_holds_on_operator_like_sums(u):
    # L(V) = lambda V + (M x M x M) V with V rank cap: factors [U, M U]
    rng = np.random.default_rng(15)
    n, cap, p = (30, 28, 26), 12, 4
    U = [_orth(rng, nk, cap) for nk in n]
    M = [np.diag(np.linspace(1.0, 1e-3, nk)) @ _orth(rng, nk, nk) for nk in n]
    core = rng.standard_normal((cap,) * 3)
    blocks = [(1e-3, O.Tucker(core, U)), (1.0, O.Tucker(core, [Mk @ Uk for Mk, Uk in zip(M, U)]))]
    s, rt = effective_sketch_size(blocks, RoundParams(eps=1e-10, cap=cap, p=p))
    assert s == cap + p and min(rt) >= cap
    assert all(shortcut(blocks, cap, tau=1e-10, u=u))


def test_holds_on_orthogonalisation_sums():
    rng = np.random.default_rng(16)
    n, cap, p = (24, 24, 24), 10, 5
    blocks = [(c, O.Tucker(rng.standard_normal((cap,) * 3), [_orth(rng, nk, cap) for nk in n]))
              for c in (1.0, -0.3, 0.05)]
    s, rt = effective_sketch_size(blocks, RoundParams(eps=1e-10, cap=cap, p=p))
    assert s == cap + p
    assert all(shortcut(blocks, cap, tau=1e-10))


def test_fails_where_the_rule_stays_below_the_cap():
    # factors confined to a dim-dimensional subspace: lambda_cap is rounding
    rng = np.random.default_rng(17)
    n, cap, p, dim = (26, 26, 26), 12, 4, 9
    B = [_orth(rng, nk, dim) for nk in n]
    blocks = [(rng.uniform(0.5, 2.0), O.Tucker(rng.standard_normal((cap,) * 3),
                                               [Bk @ rng.standard_normal((dim, cap)) for Bk in B]))
              for _ in range(4)]
    s, rt = effective_sketch_size(blocks, RoundParams(eps=1e-10, cap=cap, p=p))
    assert rt == [dim] * 3 and s == dim + p
    for u in (U64, U32):
        assert not any(shortcut(blocks, cap, tau=1e-10, u=u))


@pytest.mark.parametrize("tau", [1e-4, 1e-2])
@pytest.mark.parametrize("scale", [0.5, 2.0, 100.0])
def test_never_holds_below_the_rule(tau, scale):
    # cap - 1 unit eigenvalues and a cap-th one at scale x the rule's
    # threshold: the rule keeps it (r~ = cap) or drops it (r~ = cap - 1);
    # the shortcut may decline a kept one but never passes a dropped one
    rng = np.random.default_rng(18)
    n, cap = (40, 40, 40), 12
    Us = [_orth(rng, nk, cap) for nk in n]
    core1 = np.zeros((cap - 1,) * 3)
    for i in range(cap - 1):
        core1[i, i, i] = 1.0
    core1 /= np.linalg.norm(core1)
    tr1 = float(cap - 1)
    lam = scale * tau * tau * tr1
    blocks = [(1.0, O.Tucker(core1, [Uk[:, :cap - 1] for Uk in Us])),
              (np.sqrt(lam), O.Tucker(np.ones((1, 1, 1)), [Uk[:, cap - 1:] for Uk in Us]))]
    s, rt = effective_sketch_size(blocks, RoundParams(eps=1e-10, cap=cap, p=3, tau=tau))
    sc = shortcut(blocks, cap, tau=tau)
    for k in range(3):
        if sc[k]:
            assert rt[k] >= cap
    assert all(sc) == (scale >= 2.0)
