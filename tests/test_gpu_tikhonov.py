"""GPU parity of projected Tikhonov with GCV (Sec. 4.3) against the FP64
oracle, through the C ABI, on identical seeded inputs.

Tolerances.  At a fixed lambda everything is FP64 arithmetic on the same
data: y within max(1e-10, 100 u kappa_lambda) (relative; u the unit roundoff,
kappa_lambda = sigma_1 / max(sigma_k, lambda) the condition of the
regularised problem), the residual within 1e-12.  With lambda
chosen by GCV the choice is a continuous argmin that rounding moves where G
is flat: lambda within 1e-6 (relative), G at the GPU's lambda within 1e-9 of
the oracle's minimum, and y within the fixed-lambda bound plus the oracle's
own sensitivity ||dy/dlambda|| times the allowed lambda shift."""
import numpy as np
import pytest

import oracle as O
from oracle import tikhonov as T

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tk():
    import paper_2608_11091_amd as tk
    tk.load()
    return tk


def _graded(rng, s, k, cond):
    U, _ = np.linalg.qr(rng.standard_normal((s, k)))
    V, _ = np.linalg.qr(rng.standard_normal((k, k)))
    return U @ np.diag(np.geomspace(1.0, 1.0 / cond, k)) @ V.T


def _oracle_y_sensitivity(M, b, lam):
    # ||dy/dlambda|| by a central difference of the oracle's solution
    h = 1e-4 * lam
    yp, _, _ = T.projected_tikhonov(M, b, lam=lam + h)
    ym, _, _ = T.projected_tikhonov(M, b, lam=lam - h)
    return np.linalg.norm(yp - ym) / (2 * h)


CASES = [(1, 10, 1e2), (2, 16, 1e3), (7, 40, 1e6), (33, 120, 1e10), (64, 256, 1e12), (64, 64, 1e8)]


@pytest.mark.parametrize("k,s,cond", CASES)
def test_projected_tikhonov_parity(tk, k, s, cond):
    rng = np.random.default_rng(100 + k + s)
    M = _graded(rng, s, k, cond)
    xs = rng.standard_normal(k)
    b = M @ xs / np.linalg.norm(M @ xs) + 1e-2 * rng.standard_normal(s) / np.sqrt(s)
    Md = torch.from_numpy(M).cuda()
    bd = torch.from_numpy(b).cuda()
    print(f"projected tikhonov k={k} s={s} cond={cond:.0e}", flush=True)
    # fixed lambda: plain FP64 arithmetic on both sides
    sv = np.linalg.svd(M, compute_uv=False)
    for lam in (0.0, 1e-4, 0.1):
        y, lo, res = tk.projected_tikhonov(Md, bd, lam=lam)
        yo, reso, _ = T.projected_tikhonov(M, b, lam=lam)
        kappa = sv[0] / max(sv[-1], lam)
        if kappa > 1e8:
            continue  # the unregularised solution is as ill-conditioned as M
        assert lo == lam
        tol = max(1e-10, 100 * 1.11e-16 * kappa)
        assert np.linalg.norm(y.cpu().numpy() - yo) <= tol * np.linalg.norm(yo)
        assert abs(res - reso / np.linalg.norm(b)) <= 1e-12
    # GCV
    y, lam, res = tk.projected_tikhonov(Md, bd)
    yo, reso, lamo = T.projected_tikhonov(M, b)
    assert abs(lam / lamo - 1) <= 1e-6
    R, c, rho = T.reduce_ls(M, b)
    sig, W, bhat = T.spectral_data(R, c)
    assert T.gcv(sig, bhat, rho, lam) <= T.gcv(sig, bhat, rho, lamo) * (1 + 1e-9)
    kappa = sv[0] / max(sv[-1], lamo)
    bound = max(1e-10, 100 * 1.11e-16 * kappa) * np.linalg.norm(yo) + _oracle_y_sensitivity(M, b, lamo) * 1e-6 * lamo
    assert np.linalg.norm(y.cpu().numpy() - yo) <= bound
    assert abs(res - reso / np.linalg.norm(b)) <= 1e-8 * reso / np.linalg.norm(b) + 1e-12


def test_projected_tikhonov_zero_matrix(tk):
    # M = 0: lambda = 0, y = 0, residual ||b|| / ||b|| = 1
    Md = torch.zeros((20, 3), dtype=torch.float64, device="cuda")
    bd = torch.ones(20, dtype=torch.float64, device="cuda")
    y, lam, res = tk.projected_tikhonov(Md, bd)
    assert lam == 0.0 and float(y.abs().max()) == 0.0 and abs(res - 1.0) <= 1e-15


def _blur(n):
    from workloads import noisy_blur_problem
    K, Y, (Xc, XU), rng = noisy_blur_problem(n, 5, 0.05)
    terms = [(1.0, [K, K, K])]
    B = O.Tucker(Y, [np.eye(n) for _ in range(3)])
    return terms, B, O.Tucker(Xc, XU), rng


def _cm(Mx):
    return torch.from_numpy(np.ascontiguousarray(Mx.T)).cuda()


def _oracle_spread(run, B, reps=2, rel=1e-15):
    # the oracle's own sensitivity to unit-roundoff changes of the input: the
    # same cycle on B's core perturbed by `rel` (relative, seeded; 1e-15 for
    # the FP64 form, the FP32 unit roundoff for the FP32 form); on this
    # ill-posed problem rounding differences grow along the truncated Arnoldi
    # recurrence, so late iterations spread far more than early ones
    base = run(B)
    lam_s = np.zeros(len(base[0]))
    hist_s = np.zeros(len(base[1]))
    rre_s = x_s = 0.0
    for sd in range(reps):
        r2 = np.random.default_rng(1000 + sd)
        Bp = O.Tucker(B.core * (1 + rel * r2.standard_normal(B.core.shape)), B.U)
        lam, hist, rre, X = run(Bp)
        lam_s = np.maximum(lam_s, np.abs(lam / base[0] - 1))
        hist_s = np.maximum(hist_s, np.abs(hist / base[1] - 1))
        rre_s = max(rre_s, abs(rre / base[2] - 1))
        x_s = max(x_s, np.linalg.norm(X - base[3]) / np.linalg.norm(base[3]))
    return base, lam_s, hist_s, rre_s, x_s


@pytest.mark.parametrize("n,it", [(10, 18), (16, 24), (10, 30)])
def test_regularised_cycle_parity(tk, n, it):
    # one Alg. 2 cycle with projected Tikhonov + GCV at every iteration on a
    # noisy blur problem.  Bounds: 1e-6 (the GCV argmin's flatness), or ten
    # times the oracle's own spread under 1e-15 input changes where that is
    # larger (the later iterations of the 30-iteration case)
    terms, B, Xt, rng = _blur(n)
    cap, p, s = n, 5, 2 * it
    S = [rng.standard_normal((n, s)) for _ in range(3)]
    Om = [rng.standard_normal((n, cap + p)) for _ in range(3)]
    oprm = O.SGMRESParams(maxiter=it, k_trunc=2, cap=cap, p=p, tikhonov=True)
    xt = O.to_dense(Xt)

    def run(Bx):
        X, oi = O.sgmres_cycle(terms, Bx, S, Om, oprm, tol=1e-13)
        Xd = O.to_dense(X)
        assert oi["iters"] == it
        return np.array(oi["lam"]), np.array(oi["hist"]), np.linalg.norm(Xd - xt) / np.linalg.norm(xt), Xd

    (lo, ho, rre_o, Xo), lam_s, hist_s, rre_s, x_s = _oracle_spread(run, B)
    prm = tk.SolveParams(tol=1e-14, maxiter=it, k_trunc=2, rank_cap=cap, oversample=p, max_restarts=1,
                         tikhonov=True)
    x, info = tk.solve(tk.KronOp.from_terms(terms), tk.Tucker.from_numpy(B.core, B.U, rcap=(n,) * 3),
                       [_cm(a) for a in S], [_cm(a) for a in Om], prm)
    core, U = x.to_numpy()
    Xg = O.to_dense(O.Tucker(core, U))
    rre_g = np.linalg.norm(Xg - xt) / np.linalg.norm(xt)
    print(f"regularised cycle n={n} it={it}: gpu iters {info['iters']} rre {rre_g:.6f} lam[-1] {info['lam'][it - 1]:.4e}; "
          f"oracle rre {rre_o:.6f} lam[-1] {lo[-1]:.4e}; oracle spread lam {lam_s.max():.1e} rre {rre_s:.1e} "
          f"x {x_s:.1e}", flush=True)
    assert info["iters"] == it
    lg, hg = np.array(info["lam"][:it]), np.array(info["hist"][:it])
    assert np.all(np.abs(lg / lo - 1) <= np.maximum(1e-6, 10 * lam_s))
    assert np.all(np.abs(hg / ho - 1) <= np.maximum(1e-6, 10 * hist_s))
    assert abs(rre_g / rre_o - 1) <= max(1e-6, 10 * rre_s)
    assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) <= max(1e-6, 10 * x_s)


def test_regularised_cycle_fp32_form(tk):
    # The FP32 form (FP32 applies, TTMs, sketches and Jacobi; FP64 QR, least
    # squares and Tikhonov) against the FP64 oracle.  FP32 rounding moves the
    # sketched columns M_k by ~1e-7 relative, which the small singular values
    # of M_k (the ill-posed directions) feel at relative levels up to ~1e-3;
    # the GCV minimiser on a flat curve follows them (measured: lambda_k
    # within 20% of the oracle's, while changing only B by 2^-24 moves the
    # oracle's lambda_k by 7e-7).  What the regularisation delivers is stable:
    # the reconstruction error within 1% of the oracle's (measured 0.45%),
    # and every lambda_k within a factor 2.
    n, it = 10, 18
    terms, B, Xt, rng = _blur(n)
    cap, p, s = n, 5, 2 * it
    S = [rng.standard_normal((n, s)) for _ in range(3)]
    Om = [rng.standard_normal((n, cap + p)) for _ in range(3)]
    oprm = O.SGMRESParams(maxiter=it, k_trunc=2, cap=cap, p=p, tikhonov=True)
    xt = O.to_dense(Xt)
    Xo, oi = O.sgmres_cycle(terms, B, S, Om, oprm, tol=1e-13)
    rre_o = np.linalg.norm(O.to_dense(Xo) - xt) / np.linalg.norm(xt)
    prm = tk.SolveParams(form=1, tol=1e-14, maxiter=it, k_trunc=2, rank_cap=cap, oversample=p, max_restarts=1,
                         tikhonov=True)
    x, info = tk.solve(tk.KronOp.from_terms(terms), tk.Tucker.from_numpy(B.core, B.U, rcap=(n,) * 3),
                       [_cm(a) for a in S], [_cm(a) for a in Om], prm)
    core, U = x.to_numpy()
    rre_g = np.linalg.norm(O.to_dense(O.Tucker(core, U)) - xt) / np.linalg.norm(xt)
    ratio = np.array(info["lam"][:it]) / np.array(oi["lam"])
    print(f"regularised FP32 form: iters {info['iters']} rre {rre_g:.6f} (oracle {rre_o:.6f}); lambda ratio "
          f"[{ratio.min():.3f}, {ratio.max():.3f}]", flush=True)
    assert info["iters"] == oi["iters"] == it
    assert abs(rre_g / rre_o - 1) <= 1e-2
    assert np.all((ratio >= 0.5) & (ratio <= 2.0))


def test_regularised_mln_parity(tk):
    # MLN-Tucker sGMRES with projected Tikhonov + GCV: lambda per iteration,
    # sketched residuals and the solution, with the bounds of the cycle test
    n, r, p, it = 12, 8, 16, 20
    terms, B, Xt, rng = _blur(n)
    # rank-r compression of the noisy data (truncated HOSVD, input preparation)
    Y = O.to_dense(B)
    Q = []
    for k in range(3):
        Yk = np.moveaxis(Y, k, 0).reshape(n, -1)
        Q.append(np.linalg.svd(Yk, full_matrices=False)[0][:, :r])
    core = np.einsum("ijk,ia,jb,kc->abc", Y, Q[0], Q[1], Q[2])
    from workloads import draw_mln_sketches
    Psi = draw_mln_sketches([n] * 3, r, p, seed=11)
    oprm = O.mln.MLNParams(r=r, p=p, maxiter=it, k_trunc=2, tol=1e-14, tikhonov=True)

    def run(Bx):
        X, oi = O.mln.mln_sgmres(terms, Bx, Psi, oprm)
        assert oi["iters"] == it
        return np.array(oi["lam"]), np.array(oi["hist"]), oi["true_relres"], O.to_dense(X)

    (lo, ho, _, Xo), lam_s, hist_s, _, x_s = _oracle_spread(run, O.Tucker(core, Q))
    prm = tk.MlnParams(r=r, p=p, maxiter=it, k_trunc=2, tol=1e-14, tikhonov=True)
    x, info = tk.mln_solve(tk.KronOp.from_terms(terms), tk.Tucker.from_numpy(core, Q, rcap=(r,) * 3),
                           [_cm(a) for a in Psi], prm)
    print(f"regularised MLN: gpu iters {info['iters']} lam[-1] {info['lam'][it - 1]:.4e}; oracle lam[-1] "
          f"{lo[-1]:.4e}; oracle spread lam {lam_s.max():.1e} x {x_s:.1e}", flush=True)
    assert info["iters"] == it
    assert np.all(np.abs(np.array(info["lam"][:it]) / lo - 1) <= np.maximum(1e-6, 10 * lam_s))
    assert np.all(np.abs(np.array(info["hist"][:it]) / ho - 1) <= np.maximum(1e-6, 10 * hist_s))
    core_g, U_g = x.to_numpy()
    Xg = O.to_dense(O.Tucker(core_g, U_g))
    assert np.linalg.norm(Xg - Xo) <= max(1e-6, 10 * x_s) * np.linalg.norm(Xo)
