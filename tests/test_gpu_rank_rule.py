"""GPU parity of the Sec. 3.1 effective-rank rule at the sizes where its
Gram is wider than 160: the rule decides the sketch width s from the Gram
eigenvalues of the weighted concatenated factors, on whichever side is
smaller, at any size up to n = 512.  The oracle computes the same spectrum
with LAPACK; s must be identical and the rounded tensor within 1e-10.

Cases (each built so that the rule, not the cap, sets s):
  * n = 512, twelve rank-48 blocks (R = 576 > n): the n-side 512 x 512 Gram;
  * n = 300, five rank-40 blocks (R = 200 < n): the R-side 200 x 200 Gram;
  * n = 512 with graded block weights and tau = 0.02: the tail rule itself
    (not a numerical rank) decides, on the n-side Gram.
In all three the device's rank certificate (Courant-Fischer on the
range-finder basis, which settles r~ >= cap without the spectrum) is tried
and must decline: r~ < cap.  The last case guards its tau^2 term: with the
zero clamp alone the certificate would pass there.

The certificate is planned for every FP64 RoundSum and, in the FP32 form,
for the sums whose Gram can exceed the register eigensolver's order 160
(elsewhere the FP32 spectrum is cheaper than the certificate and runs beside
the range sketch).  Cases where it must pass (r~ >= cap, s = cap + p), with s
identical to the oracle's:
  * the operator sum lambda V + (M x M x M) V at n = 512, cap 48 (factors
    [U, M U]: the RoundSum of every sGMRES iteration), FP64; in FP32 (Gram
    order 96) the spectrum path runs and no certificate is tried;
  * a sixty-block sum (the final assembly of a 60-iteration cycle), where
    the rule would otherwise need the 512 x 512 n-side spectrum, FP64 and
    FP32."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tk():
    import paper_2608_11091_amd as tk
    tk.load()
    return tk


def _cm(M):
    return torch.from_numpy(np.ascontiguousarray(M.T)).cuda()


def _dist(A, B):
    return O.exact_norm([(1.0, A), (-1.0, B)]) / O.exact_norm([(1.0, B)])


def _subspace_blocks(rng, n, nb, r, dim):
    """nb blocks of rank r whose mode-k factors lie in a fixed dim-dimensional
    subspace: the concatenation has numerical rank dim in every mode."""
    B = [np.linalg.qr(rng.standard_normal((nk, dim)))[0] for nk in n]
    out = []
    for _ in range(nb):
        U = [Bk @ rng.standard_normal((dim, r)) for Bk in B]   # rank dim < r
        core = rng.standard_normal((r,) * len(n)) * rng.uniform(0.5, 2.0)
        out.append((float(rng.uniform(-1.5, 1.5)), O.Tucker(core, U)))
    return out


def _run(tk, blocks, cap, p, eps, tau=None, form=0, expect_cert=False, expect_tried=True):
    n = blocks[0][1].n
    rng = np.random.default_rng(99)
    Om = [rng.standard_normal((nk, cap + p)) for nk in n]
    prm = O.RoundParams(eps=eps, cap=cap, p=p, tau=tau)
    Xo, info = O.roundsum(blocks, Om, prm)
    gb = [(c, tk.Tucker.from_numpy(X.core, X.U, rcap=(X.core.shape[0],) * len(n))) for c, X in blocks]
    t0, p0 = tk.rank_cert_count()
    Xg, s = tk.rhosvd(gb, [_cm(o) for o in Om], eps=eps, cap=cap, p=p, tau=-1.0 if tau is None else tau, form=form)
    t1, p1 = tk.rank_cert_count()
    print("oracle s", info["s"], "r~", info["rtilde"], "ranks", info["ranks"], "| gpu s", s, "ranks", Xg.ranks,
          "| certificates tried", t1 - t0, "passed", p1 - p0, flush=True)
    assert t1 - t0 == (len(n) if expect_tried else 0)   # one check per mode
    assert (p1 - p0 > 0) == expect_cert
    return Xo, info, Xg, s


def test_rank_rule_nside_512(tk):
    rng = np.random.default_rng(21)
    blocks = _subspace_blocks(rng, (512, 512, 512), nb=12, r=48, dim=40)
    Xo, info, Xg, s = _run(tk, blocks, cap=48, p=5, eps=1e-10)
    assert info["rtilde"] == [40, 40, 40] and info["s"] == 45   # the rule, not the cap, sets s
    assert s == info["s"] and list(Xg.ranks) == list(info["ranks"])
    Xc = O.Tucker(*Xg.to_numpy())
    assert _dist(Xc, Xo) <= 1e-10


def test_rank_rule_rside_200(tk):
    rng = np.random.default_rng(22)
    blocks = _subspace_blocks(rng, (300, 310, 300), nb=5, r=40, dim=30)
    Xo, info, Xg, s = _run(tk, blocks, cap=40, p=5, eps=1e-10)
    assert info["rtilde"] == [30, 30, 30] and info["s"] == 35
    assert s == info["s"] and list(Xg.ranks) == list(info["ranks"])
    assert _dist(O.Tucker(*Xg.to_numpy()), Xo) <= 1e-10


def test_rank_rule_tail_threshold_512(tk):
    rng = np.random.default_rng(23)
    n = (512, 512, 512)
    blocks = []
    for b in range(14):
        U = [np.linalg.qr(rng.standard_normal((nk, 8)))[0] for nk in n]
        core = rng.standard_normal((8, 8, 8))
        core *= 10.0 ** (-0.35 * b) / np.linalg.norm(core)
        blocks.append((1.0, O.Tucker(core, U)))
    Xo, info, Xg, s = _run(tk, blocks, cap=56, p=5, eps=1e-10, tau=0.02)
    assert max(info["rtilde"]) + 5 < 61            # below the capped width
    assert s == info["s"]
    assert list(Xg.ranks) == list(info["ranks"])
    assert _dist(O.Tucker(*Xg.to_numpy()), Xo) <= 1e-10


def _operator_sum(rng, n, cap, lam=1e-3):
    U = [np.linalg.qr(rng.standard_normal((nk, cap)))[0] for nk in n]
    M = []
    for nk in n:
        Q = np.linalg.qr(rng.standard_normal((nk, nk)))[0]
        M.append((Q * np.linspace(1.0, 1e-4, nk)) @ Q.T)
    core = rng.standard_normal((cap,) * len(n))
    return [(lam, O.Tucker(core, U)), (1.0, O.Tucker(core, [Mk @ Uk for Mk, Uk in zip(M, U)]))]


@pytest.mark.parametrize("form", [0, 1])
def test_rank_certificate_operator_sum_512(tk, form):
    rng = np.random.default_rng(24)
    blocks = _operator_sum(rng, (512, 512, 512), cap=48)
    Xo, info, Xg, s = _run(tk, blocks, cap=48, p=5, eps=1e-10, form=form, expect_cert=form == 0,
                           expect_tried=form == 0)
    assert info["s"] == 53 and s == 53
    assert list(Xg.ranks) == list(info["ranks"])
    Xc = O.Tucker(*Xg.to_numpy())
    assert _dist(Xc, Xo) <= (1e-10 if form == 0 else 1e-5)


@pytest.mark.parametrize("form", [0, 1])
def test_rank_certificate_sixty_blocks_512(tk, form):
    # sixty orthonormal rank-48 blocks with decaying coefficients, as in the
    # final assembly sum_i y_i V_i of a 60-iteration cycle (R = 2880 > n)
    rng = np.random.default_rng(25)
    n, cap = (512, 512, 512), 48
    blocks = []
    for i in range(60):
        U = [np.linalg.qr(rng.standard_normal((nk, cap)))[0] for nk in n]
        core = rng.standard_normal((cap,) * 3)
        blocks.append((float(0.8 ** i * rng.choice([-1.0, 1.0])), O.Tucker(core / np.linalg.norm(core), U)))
    Xo, info, Xg, s = _run(tk, blocks, cap=cap, p=5, eps=1e-10, form=form, expect_cert=True)
    assert info["s"] == 53 and s == 53
    assert list(Xg.ranks) == list(info["ranks"])
    assert _dist(O.Tucker(*Xg.to_numpy()), Xo) <= (1e-10 if form == 0 else 1e-5)
