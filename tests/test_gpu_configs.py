"""Solve parity on the convection-diffusion workload (d = 3, n = 256, six
Kronecker terms, rank cap 32) in both forms, and the forward and adjoint
solves of the 4D workload (d = 4, n = 128, Poisson plus a rank-2 perturbation,
rank cap 32, k_trunc 3) in the FP32 form, each over one restart cycle against
the FP64 oracle on identical seeded inputs.

Bounds are measured (_spread.py).  FP64 form: every sketched residual, the
cycle's true residual and its solution within ten times the largest spread of
the oracle over a one-ulp change of the right-hand side and over the
range-finder basis choice, and of the GPU's own solve under a one-ulp change
(at least 1e-10).  FP32 form: the iterations before the rank cap binds
within the FP32 RoundSum bound 1e-4, a non-increasing sketched residual, and
the cycle's true residual and solution within ten times the largest spread of
the oracle runs above, the oracle run with every operand rounded to FP32 and
the GPU's own FP32 solve under an FP32-level change of the right-hand side
(at least 1e-4)."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from workloads import make_config

from _spread import (bound_from_spreads, cholesky_qr3, first_divergence, fp32_operands, history_bound,
                     perturbed_rhs, rel_spread)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
FP32_FLOOR = 1e-4


@pytest.fixture(scope="module")
def tk():
    import paper_2608_11091_amd as tk
    tk.load()
    return tk


def _cm(M):
    return torch.from_numpy(np.ascontiguousarray(M.T)).cuda()


def _cpu(tk, X):
    return O.Tucker(*X.to_numpy())


def _dist(A, B):
    return O.exact_norm([(1.0, A), (-1.0, B)]) / O.exact_norm([(1.0, B)])


def _hist(log):
    return np.array([e["res"] for e in log if "k" in e])


def _ensemble(terms, B, S, Om, oprm, fp32=False):
    """Reference oracle run plus its valid rounding-level variants."""
    out = {}
    log = []
    X, info = O.solve(terms, B, S, Om, oprm, log=log)
    out["ref"] = (X, info, _hist(log), [tuple(e["r2"]) for e in log if "k" in e])
    variants = [("ulp", (terms, perturbed_rhs(B), S, Om), oprm),
                ("basis", (terms, B, S, Om), dataclasses.replace(oprm, range_basis=cholesky_qr3))]
    if fp32:
        from _spread import f32
        variants.append(("fp32", fp32_operands(terms, B, S, Om), dataclasses.replace(oprm, operand_rounding=f32)))
    for key, args, prm in variants:
        log = []
        X, info = O.solve(*args, prm, log=log)
        out[key] = (X, info, _hist(log), None)
    return out


@pytest.fixture(scope="module")
def convdiff():
    w = make_config(2)
    B = O.Tucker(w.b_core, w.b_factors)
    oprm = O.SGMRESParams(tol=w.tol, eta=w.eta, maxiter=w.maxiter, max_restarts=1, k_trunc=w.k_trunc, cap=w.cap,
                          p=w.p)
    return w, _ensemble(w.terms, B, w.S, w.Omega, oprm, fp32=True)


@pytest.mark.parametrize("form", [0, 1])
def test_convdiff_cycle(tk, convdiff, form):
    w, ens = convdiff
    Xo, oi, h_o, ro = ens["ref"]
    prm = tk.SolveParams(form=form, tol=w.tol, eta=w.eta, maxiter=w.maxiter, max_restarts=1, k_trunc=w.k_trunc,
                         rank_cap=w.cap, oversample=w.p)
    op = tk.KronOp.from_terms(w.terms)
    S, Om = [_cm(s) for s in w.S], [_cm(o) for o in w.Omega]
    x, info = tk.solve(op, tk.Tucker.from_numpy(w.b_core, w.b_factors), S, Om, prm)
    # the GPU's own spread: the same solve on the right-hand side changed by
    # one unit roundoff of the form
    Bp = perturbed_rhs(O.Tucker(w.b_core, w.b_factors), rel=2.0 ** -52 if form == 0 else U32)
    xp, ip = tk.solve(op, tk.Tucker.from_numpy(Bp.core, Bp.U), S, Om, prm)
    h_g = np.array(info["hist"])
    m = min(len(h_g), len(h_o))
    dev = np.abs(h_g[:m] - h_o[:m]) / h_o[:m]
    X = _cpu(tk, x)
    dev_x = _dist(X, Xo)
    dev_t = abs(info["true_relres"] / oi["true_relres"] - 1.0)
    g_h = rel_spread(h_g, ip["hist"])
    g_x = _dist(_cpu(tk, xp), X)
    g_t = abs(ip["true_relres"] / info["true_relres"] - 1.0)
    keys = ["ulp", "basis"] if form == 0 else ["ulp", "basis", "fp32"]
    sx = max(_dist(ens[k][0], Xo) for k in keys)
    st = max(abs(ens[k][1]["true_relres"] / oi["true_relres"] - 1.0) for k in keys)
    sx, st = max(sx, g_x), max(st, g_t)
    spreads = [rel_spread(h_o, ens[k][2]) for k in keys] + [g_h]
    if form == 0:
        floor = 1e-10
        bound = bound_from_spreads(spreads, m, floor)
    else:
        # FP32: per iteration only before the rank cap binds (no truncation
        # inside a singular-value continuum yet, nothing amplified); after
        # that, the end of the cycle
        calm = np.array([max(r) < w.cap for r in ro])
        assert calm[:3].all()
        floor = FP32_FLOOR
        bound = np.where(calm[:m], FP32_FLOOR, np.inf)
        assert np.all(np.diff(h_g) <= 1e-6 * h_g[:-1])    # the sketched residual never increases
    print(f"convdiff n=256 form {form}: iters gpu {info['iters']} oracle {oi['iters']}; first divergence above "
          f"{floor:g} at {first_divergence(h_g, h_o, floor)}; sketched dev max {dev.max():.2e} (worst ratio to the "
          f"bound {np.max(dev / bound[:m]):.2f}); true residual {info['true_relres']:.4e} "
          f"vs {oi['true_relres']:.4e} (dev {dev_t:.2e}, spread {st:.2e}); solution dev {dev_x:.2e} "
          f"(spread {sx:.2e})", flush=True)
    assert info["iters"] == oi["iters"]
    if form == 0:
        assert info["ranks"] == ro
    assert np.all(dev <= bound[:m]), np.nonzero(dev > bound[:m])[0]
    assert dev_t <= max(floor, 10 * st)
    assert dev_x <= max(floor, 10 * sx)


def test_poisson4d_forward_and_adjoint_fp32(tk):
    # Five iterations of one cycle keep the d = 4 oracle (32^4 cores) within
    # a minute; the adjoint solve's right-hand side is a random rank-(4,4,4,4)
    # Tucker tensor.  In five iterations the trajectory stays calm (no
    # amplification yet), so every result is held to the FP32 RoundSum bound
    # 1e-4 or ten times the FP32-operand oracle's spread, whichever is larger.
    from _spread import f32
    it = 5
    w = make_config(5)
    B = O.Tucker(w.b_core, w.b_factors)
    rng = np.random.default_rng(55)
    Xbar = O.Tucker(rng.standard_normal((4,) * 4), [rng.standard_normal((128, 4)) for _ in range(4)])
    kw = dict(tol=w.tol, eta=w.eta, maxiter=it, max_restarts=1, k_trunc=w.k_trunc)
    oprm = O.SGMRESParams(cap=w.cap, p=w.p, **kw)
    oprm32 = dataclasses.replace(oprm, operand_rounding=f32)
    S, Om = [_cm(s) for s in w.S], [_cm(o) for o in w.Omega]
    op = tk.KronOp.from_terms(w.terms)
    prm = tk.SolveParams(form=1, rank_cap=w.cap, oversample=w.p, **kw)
    # forward
    log, log32 = [], []
    Xo, oi = O.solve(w.terms, B, w.S, w.Omega, oprm, log=log)
    X32, i32 = O.solve(*fp32_operands(w.terms, B, w.S, w.Omega), oprm32, log=log32)
    x, info = tk.solve(op, tk.Tucker.from_numpy(w.b_core, w.b_factors), S, Om, prm)
    h_o, h_g = _hist(log), np.array(info["hist"])
    bound = history_bound(h_o, [_hist(log32)], floor=FP32_FLOOR)
    dev = np.abs(h_g - h_o) / h_o
    dev_x, spread_x = _dist(_cpu(tk, x), Xo), _dist(X32, Xo)
    print(f"poisson4d forward fp32: sketched dev {dev} (bound {bound}); true residual {info['true_relres']:.6e} vs "
          f"{oi['true_relres']:.6e}; solution dev {dev_x:.2e} (fp32-operand spread {spread_x:.2e})", flush=True)
    assert info["iters"] == oi["iters"] == it
    assert np.all(dev <= bound), np.nonzero(dev > bound)[0]
    assert dev_x <= max(FP32_FLOOR, 10 * spread_x)
    assert abs(info["true_relres"] / oi["true_relres"] - 1.0) <= FP32_FLOOR
    # adjoint: L^T lambda = xbar and dl/dalpha_j = -<lambda, x x_k A_j^(k)> at the GPU's forward solution
    Xg = _cpu(tk, x)
    lam_o, dal_o, _, li = O.adjoint_gradients(w.terms, Xg, [(1.0, Xbar)], w.S, w.Omega, oprm, want_dA=False)
    t32, _, S32, O32 = fp32_operands(w.terms, B, w.S, w.Omega)
    Xb32 = O.Tucker(f32(Xbar.core), [f32(u) for u in Xbar.U])
    lam_p, dal_p, _, _ = O.adjoint_gradients(t32, Xg, [(1.0, Xb32)], S32, O32, oprm32, want_dA=False)
    xg = tk.Tucker.from_numpy(Xg.core, Xg.U)
    lam_g, dal_g, _, bi = tk.backward(op, xg, [(1.0, tk.Tucker.from_numpy(Xbar.core, Xbar.U))], S, Om, prm,
                                      want_dA=False)
    dev_l, spread_l = _dist(_cpu(tk, lam_g), lam_o), _dist(lam_p, lam_o)
    dev_a = np.abs(dal_g - dal_o) / np.abs(dal_o)
    spread_a = np.abs(dal_p - dal_o) / np.abs(dal_o)
    print(f"poisson4d adjoint fp32: lambda dev {dev_l:.2e} (spread {spread_l:.2e}); dalpha dev {dev_a} "
          f"(spread {spread_a}); adjoint true residual {bi['true_relres']:.6e} vs {li['true_relres']:.6e}",
          flush=True)
    assert bi["iters"] == li["iters"] == it
    assert dev_l <= max(FP32_FLOOR, 10 * spread_l)
    assert np.all(dev_a <= np.maximum(FP32_FLOOR, 10 * spread_a))
