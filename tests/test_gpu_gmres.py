"""GPU parity of RHOSVD-Tucker GMRES (Alg. 1, full Arnoldi) against the FP64
oracle, through the C ABI, on identical seeded inputs.  Bounds as for the
sketched cycle: first-cycle residual histories (fractions of ||B||) within
the FP64 parity bound 1e-10, equal iteration counts and per-iteration ranks,
the true residuals of the cycle solutions within 1e-10 of each other and the
refined solutions at the tolerance;
the regularised run within 1e-6 or ten times the oracle's own spread."""
import numpy as np
import pytest

import oracle as O
from oracle.gmres import gmres_cycle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tk():
    import paper_2608_11091_amd as tk
    tk.load()
    return tk


def _cm(Mx):
    return torch.from_numpy(np.ascontiguousarray(Mx.T)).cuda()


@pytest.mark.parametrize("n,cap,it", [(32, 16, 40), (24, 24, 30)])
def test_gmres_cycle_parity(tk, n, cap, it):
    from workloads import make_config
    w = make_config(1, n=n, cap=cap)
    B = O.Tucker(w.b_core, w.b_factors)
    oprm = O.SGMRESParams(maxiter=it, cap=cap, p=w.p)
    log = []
    Xo, oi = gmres_cycle(w.terms, B, w.Omega, oprm, tol=1e-9, log=log)
    prm = tk.SolveParams(form=0, tol=1e-9, maxiter=it, rank_cap=cap, oversample=w.p, max_restarts=1, method=1)
    x, info = tk.solve(tk.KronOp.from_terms(w.terms), tk.Tucker.from_numpy(w.b_core, w.b_factors, rcap=(cap,) * 3),
                       None, [_cm(a) for a in w.Omega], prm)
    print(f"gmres cycle n={n} cap={cap}: gpu iters {info['iters']} last {info['hist'][-1]:.3e}; oracle iters "
          f"{oi['iters']} last {oi['hist'][-1]:.3e}", flush=True)
    assert info["iters"] == oi["iters"]
    its = [e for e in log if "k" in e]
    assert [tuple(e["r2"]) for e in its] == info["ranks"][:oi["iters"]]
    assert np.max(np.abs(np.array(info["hist"][:oi["iters"]]) - np.array(oi["hist"]))) <= 1e-10
    # the true residuals of both cycle solutions, evaluated by the oracle,
    # agree to the parity bound (fractions of ||B||)
    core, U = x.to_numpy()
    Xg = O.Tucker(core, U)
    bn = O.exact_norm([(1.0, B)])
    res = [O.exact_norm([(1.0, B)] + [(-c, T) for c, T in O.apply_op(w.terms, X)]) / bn for X in (Xg, Xo)]
    assert abs(res[0] - res[1]) <= 1e-10


def test_gmres_restarted_solve_nonsymmetric(tk):
    # convection-diffusion in Kronecker-sum form (6 terms) at n = 16, refined
    # to 1e-10: equal status, iterations and cycles; the GPU solution's true
    # residual, checked by the oracle, at the tolerance
    from workloads import make_config
    w = make_config(2, n=16, cap=16)
    B = O.Tucker(w.b_core, w.b_factors)
    oprm = O.SGMRESParams(tol=1e-10, maxiter=40, cap=16, p=w.p, max_restarts=6)
    Xo, oi = O.solve(w.terms, B, None, w.Omega, oprm, method="gmres")
    prm = tk.SolveParams(form=0, tol=1e-10, maxiter=40, rank_cap=16, oversample=w.p, max_restarts=6, method=1)
    x, info = tk.solve(tk.KronOp.from_terms(w.terms), tk.Tucker.from_numpy(w.b_core, w.b_factors, rcap=(16,) * 3),
                       None, [_cm(a) for a in w.Omega], prm)
    print(f"gmres convdiff n=16: gpu {info['status_name']} iters {info['iters']} cycles {info['cycles']} true "
          f"{info['true_relres']:.3e}; oracle {oi['status']} iters {oi['iters']} cycles {oi['cycles']} true "
          f"{oi['true_relres']:.3e}", flush=True)
    assert info["status"] == oi["status"] == 0
    assert info["iters"] == oi["iters"] and info["cycles"] == oi["cycles"]
    core, U = x.to_numpy()
    X = O.Tucker(core, U)
    rel = O.exact_norm([(1.0, B)] + [(-c, T) for c, T in O.apply_op(w.terms, X)]) / O.exact_norm([(1.0, B)])
    assert rel <= 1e-10


def test_gmres_fp32_form_reaches_tolerance(tk):
    # FP32 full-Arnoldi cycles inside the FP64 refinement reach 1e-8
    from workloads import make_config
    w = make_config(1, n=16, cap=16)
    prm = tk.SolveParams(form=1, tol=1e-8, maxiter=40, rank_cap=16, oversample=w.p, max_restarts=8, method=1)
    x, info = tk.solve(tk.KronOp.from_terms(w.terms), tk.Tucker.from_numpy(w.b_core, w.b_factors, rcap=(16,) * 3),
                       None, [_cm(a) for a in w.Omega], prm)
    print(f"gmres fp32 form: {info['status_name']} iters {info['iters']} cycles {info['cycles']} true "
          f"{info['true_relres']:.3e}", flush=True)
    assert info["status"] == 0
    B = O.Tucker(w.b_core, w.b_factors)
    core, U = x.to_numpy()
    rel = O.exact_norm([(1.0, B)] + [(-c, T) for c, T in O.apply_op(w.terms, O.Tucker(core, U))]) / \
        O.exact_norm([(1.0, B)])
    assert rel <= 1e-8


def test_gmres_tikhonov_parity(tk):
    # projected Tikhonov + GCV on the Hessenberg problem (Sec. 4.3) on the
    # noisy blur problem of the sketched tests
    from test_gpu_tikhonov import _blur, _oracle_spread
    n, it = 10, 18
    terms, B, Xt, rng = _blur(n)
    Om = [rng.standard_normal((n, n + 5)) for _ in range(3)]
    oprm = O.SGMRESParams(maxiter=it, cap=n, p=5, tikhonov=True)
    xt = O.to_dense(Xt)

    def run(Bx):
        X, oi = gmres_cycle(terms, Bx, Om, oprm, tol=1e-13)
        Xd = O.to_dense(X)
        assert oi["iters"] == it
        return np.array(oi["lam"]), np.array(oi["hist"]), np.linalg.norm(Xd - xt) / np.linalg.norm(xt), Xd

    (lo, ho, rre_o, Xo), lam_s, hist_s, rre_s, x_s = _oracle_spread(run, B)
    prm = tk.SolveParams(tol=1e-14, maxiter=it, rank_cap=n, oversample=5, max_restarts=1, tikhonov=True, method=1)
    x, info = tk.solve(tk.KronOp.from_terms(terms), tk.Tucker.from_numpy(B.core, B.U, rcap=(n,) * 3), None,
                       [_cm(a) for a in Om], prm)
    core, U = x.to_numpy()
    Xg = O.to_dense(O.Tucker(core, U))
    print(f"gmres tikhonov: gpu iters {info['iters']} lam[-1] {info['lam'][it - 1]:.4e}; oracle lam[-1] "
          f"{lo[-1]:.4e}; spread lam {lam_s.max():.1e} x {x_s:.1e}", flush=True)
    assert info["iters"] == it
    assert np.all(np.abs(np.array(info["lam"][:it]) / lo - 1) <= np.maximum(1e-6, 10 * lam_s))
    assert np.all(np.abs(np.array(info["hist"][:it]) / ho - 1) <= np.maximum(1e-6, 10 * hist_s))
    assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) <= max(1e-6, 10 * x_s)
