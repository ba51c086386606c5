"""BF16-factor form of the per-call entry points against the FP64 oracle on
identical seeded inputs, at the full workload sizes.  In this form every
product with a Tucker factor rounds both operands to bfloat16 (unit roundoff
u_b = 2^-8, round to nearest even) and accumulates in FP32 on the BF16
matrix cores; cores, Grams, QRs and eigensolves keep the FP32 form's
arithmetic.  Per-result bounds:

* factor products A U (Eq. (2)): rounding both operands perturbs each
  product term by at most (2 u_b + u_b^2) |a||u|, and the FP32 sum of n terms
  adds n u |a||u|, so ||P_b - P||_F <= (2 u_b + u_b^2 + n u) ||A||_F ||U||_F;
  and, as a stated per-result target, a relative error <= 1e-2;
* Khatri-Rao sketch of L(X): relative error <= 1e-2;
* RoundSum of L(X) with the oracle's sketch width and ranks replayed
  (Sec. 3.1): Tucker distance <= 3e-2.
The solver runs in FP64 or FP32 only: a BF16 solve is rejected."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

UB = 2.0 ** -8
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
def test_bf16_bounds(tk, cfg):
    from workloads import make_config
    w = make_config(cfg)
    rng = np.random.default_rng(40 + cfg)
    X = _basis_like(rng, w.n, w.cap)
    op = tk.KronOp.from_terms(w.terms)
    Xg = tk.Tucker.from_numpy(X.core, X.U)
    ref = O.apply_op(w.terms, X)
    got = tk.apply_op(op, Xg, form=2)
    got32 = tk.apply_op(op, Xg, form=1)
    assert len(ref) == len(got) == len(w.terms)
    for (_, fs), (_, A_), (_, B_), (_, C_) in zip(w.terms, ref, got, got32):
        Bc, Cc = _cpu(B_), _cpu(C_)
        for k in range(w.d):
            if fs[k] is None:
                continue
            err = np.linalg.norm(Bc.U[k] - A_.U[k])
            rel = err / np.linalg.norm(A_.U[k])
            err32 = np.linalg.norm(Cc.U[k] - A_.U[k])
            bound = (2 * UB + UB * UB + w.n[k] * U32) * np.linalg.norm(fs[k]) * np.linalg.norm(X.U[k])
            print(f"apply cfg{cfg} mode {k}: bf16 error {err:.2e} (relative {rel:.2e}, bound {bound:.2e}); "
                  f"fp32 error {err32:.2e}", flush=True)
            assert err <= bound, (k, err, bound)
            assert rel <= 1e-2, (k, rel)
            # the BF16 products are BF16 products: far less accurate than FP32
            assert err > 10 * err32
    s64 = O.sketch_krp(ref, w.S)
    sb = tk.sketch(got, [_cm(s) for s in w.S], form=2).cpu().numpy()
    rel_s = np.linalg.norm(sb - s64) / np.linalg.norm(s64)
    print(f"sketch cfg{cfg}: relative error {rel_s:.2e}", flush=True)
    assert rel_s <= 1e-2
    Xo, info = O.roundsum(ref, w.Omega, O.RoundParams(eps=1e-6, cap=w.cap, p=w.p))
    got64 = tk.apply_op(op, Xg)
    Wg, s = tk.rhosvd(got64, [_cm(o) for o in w.Omega], eps=1e-6, cap=w.cap, p=w.p, force_s=info["s"],
                      force_ranks=list(info["ranks"]), form=2)
    assert s == info["s"] and list(Wg.ranks) == list(info["ranks"])
    dist = O.exact_norm([(1.0, _cpu(Wg)), (-1.0, Xo)]) / O.exact_norm([(1.0, Xo)])
    print(f"RoundSum cfg{cfg}: distance {dist:.2e} (s {s}, ranks {list(Wg.ranks)})", flush=True)
    assert dist <= 3e-2, dist


def test_bf16_solve_is_rejected(tk):
    from workloads import laplacian_1d
    n, cap, p = 16, 8, 3
    L = laplacian_1d(n)
    op = tk.KronOp.from_terms([(1.0, [L if j == k else None for j in range(3)]) for k in range(3)])
    b = tk.Tucker.from_numpy(np.ones((1, 1, 1)), [np.ones((n, 1))] * 3, rcap=(cap,) * 3)
    rng = np.random.default_rng(1)
    S = [_cm(rng.standard_normal((n, 40))) for _ in range(3)]
    Om = [_cm(rng.standard_normal((n, cap + p))) for _ in range(3)]
    with pytest.raises(tk.TkError) as e:
        tk.solve(op, b, S, Om, tk.SolveParams(form=2, tol=1e-8, maxiter=10, rank_cap=cap, oversample=p))
    assert e.value.code == -7
