"""Reduced-precision parity: the FP32 form of each per-call entry point
against the FP64 oracle on identical seeded inputs, at the full workload
sizes, to the per-result bounds of FP32 arithmetic (unit roundoff
u = 2^-24, FP32 accumulation on the matrix cores):

* factor products A U (Eq. (2)):   ||P32 - P||_F <= 2 sqrt(n) u ||A||_F ||U||_F
  (inputs rounded to FP32, then a length-n inner product per entry);
* Khatri-Rao sketch of L(X):        ||s32 - s|| <= 1e-5 ||s||;
* RoundSum of L(X) with the oracle's sketch width and ranks replayed
  (Sec. 3.1; FP64 range-sketch QR, everything else FP32): Tucker distance
  <= 1e-4, for a sum whose singular values decay geometrically, so that the
  cut at the rank cap falls into a gap rather than a cluster.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def tk():
    import paper_2608_11091_amd as tk
    tk.load()
    return tk


def _cm(M):
    return torch.from_numpy(np.ascontiguousarray(M.T)).cuda()


def _cpu(X):
    core, U = X.to_numpy()
    return O.Tucker(core, U)


def _basis_like(rng, n, r):
    d = len(n)
    U = [np.linalg.qr(rng.standard_normal((nk, r)))[0] for nk in n]
    core = rng.standard_normal((r,) * d)
    w = 0.8 ** np.arange(r)
    for k in range(d):
        shape = [1] * d
        shape[k] = r
        core = core * w.reshape(shape)
    core /= np.linalg.norm(core)
    return O.Tucker(core, U)


@pytest.mark.parametrize("cfg", [3, 2, 5])
def test_fp32_bounds(tk, cfg):
    from workloads import make_config
    w = make_config(cfg)
    rng = np.random.default_rng(30 + cfg)
    X = _basis_like(rng, w.n, w.cap)
    op = tk.KronOp.from_terms(w.terms)
    Xg = tk.Tucker.from_numpy(X.core, X.U)
    # factor products
    ref = O.apply_op(w.terms, X)
    got = tk.apply_op(op, Xg, form=1)
    assert len(ref) == len(got) == len(w.terms)
    for (_, fs), (_, A_), (_, B_) in zip(w.terms, ref, got):
        Bc = _cpu(B_)
        for k in range(w.d):
            if fs[k] is None:
                continue
            err = np.linalg.norm(Bc.U[k] - A_.U[k])
            bound = 2 * np.sqrt(w.n[k]) * U32 * np.linalg.norm(fs[k]) * np.linalg.norm(X.U[k])
            print(f"apply cfg{cfg} mode {k}: error {err:.2e}, bound {bound:.2e}")
            assert err <= bound, (k, err, bound)
    # sketch of L(X)
    s64 = O.sketch_krp(ref, w.S)
    s32 = tk.sketch(got, [_cm(s) for s in w.S], form=1).cpu().numpy()
    rel_s = np.linalg.norm(s32 - s64) / np.linalg.norm(s64)
    print(f"sketch cfg{cfg}: relative error {rel_s:.2e}")
    assert rel_s <= 1e-5
    # RoundSum of L(X) with the oracle's decisions replayed
    Xo, info = O.roundsum(ref, w.Omega, O.RoundParams(eps=1e-6, cap=w.cap, p=w.p))
    got64 = tk.apply_op(op, Xg)   # FP64 inputs, so that only the RoundSum runs in FP32
    Wg, s = tk.rhosvd(got64, [_cm(o) for o in w.Omega], eps=1e-6, cap=w.cap, p=w.p, force_s=info["s"],
                      force_ranks=list(info["ranks"]), form=1)
    assert s == info["s"] and list(Wg.ranks) == list(info["ranks"])
    Wc = _cpu(Wg)
    dist = O.exact_norm([(1.0, Wc), (-1.0, Xo)]) / O.exact_norm([(1.0, Xo)])
    print(f"RoundSum cfg{cfg}: distance {dist:.2e} (s {s}, ranks {list(Wg.ranks)})")
    assert dist <= 1e-4, dist
