"""The torch.autograd.Function around the hand-written adjoint
(TuckerSGMRESLoss), driven by torch.autograd.backward: the gradients with
respect to the operator coefficients alpha (a CUDA tensor) and the core of the
right-hand side b are checked against the oracle's adjoint (1e-8), against
the dense FP64 gradient of the tiny problem (N = 1000) and against central
finite differences of forward solves.  A solve that does not converge raises."""
import numpy as np
import pytest

import oracle as O
from workloads import laplacian_1d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tk():
    import paper_2608_11091_amd as tk
    tk.load()
    return tk


def _cm(M):
    return torch.from_numpy(np.ascontiguousarray(M.T)).cuda()


def _problem(tk, n=10, seed=7, tol=1e-12, maxiter=40, max_restarts=50):
    rng = np.random.default_rng(seed)
    L = laplacian_1d(n)
    theta = [0.8, 1.4, 0.6]
    terms = [(theta[k], [L if j == k else None for j in range(3)]) for k in range(3)]
    B = O.Tucker(rng.standard_normal((2, 2, 2)), [rng.standard_normal((n, 2)) for _ in range(3)])
    Xt = O.Tucker(rng.standard_normal((2, 2, 2)), [rng.standard_normal((n, 2)) for _ in range(3)])
    S = [rng.standard_normal((n, 80)) for _ in range(3)]
    Om = [rng.standard_normal((n, 15)) for _ in range(3)]
    oprm = O.SGMRESParams(tol=tol, maxiter=maxiter, k_trunc=2, cap=n, p=5, max_restarts=max_restarts)
    prm = tk.SolveParams(form=0, tol=tol, maxiter=maxiter, k_trunc=2, rank_cap=n, oversample=5,
                         max_restarts=max_restarts)
    problem = dict(op=tk.KronOp.from_terms(terms), b=tk.Tucker.from_numpy(B.core, B.U),
                   x_target=tk.Tucker.from_numpy(Xt.core, Xt.U), S=[_cm(s) for s in S], omega=[_cm(o) for o in Om],
                   prm=prm)
    return terms, theta, B, Xt, S, Om, oprm, problem


def _loss(tk, alpha, b_core, problem):
    return tk.TuckerSGMRESLoss.apply(alpha, b_core, problem)


def test_autograd_gradients_against_oracle_dense_and_fd(tk):
    n = 10
    terms, theta, B, Xt, S, Om, oprm, problem = _problem(tk, n)
    alpha = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
    b_core = torch.tensor(B.core, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = _loss(tk, alpha, b_core, problem)
    torch.autograd.backward(loss)
    assert alpha.grad is not None and alpha.grad.device == alpha.device and alpha.grad.dtype == torch.float64
    assert b_core.grad is not None and b_core.grad.shape == b_core.shape and b_core.grad.device == b_core.device
    ga = alpha.grad.cpu().numpy()
    gb = b_core.grad.cpu().numpy()
    # the oracle's adjoint
    x, _ = O.solve(terms, B, S, Om, oprm)
    lo, xbar = O.loss_and_cotangent(x, Xt)
    lam, dalpha, _, _ = O.adjoint_gradients(terms, x, xbar, S, Om, oprm, want_dA=False)
    dcore = O.multi_ttm(lam.core, [B.U[k].T @ lam.U[k] for k in range(3)])
    print("loss", float(loss.detach()), lo, "dalpha", ga, dalpha, flush=True)
    assert abs(float(loss.detach()) / lo - 1.0) <= 1e-8
    assert np.allclose(ga, dalpha, rtol=1e-8, atol=0)
    assert np.linalg.norm(gb - dcore) <= 1e-8 * np.linalg.norm(dcore)
    # the dense FP64 gradient (N = 1000, row-major vec)
    A = O.dense_operator(terms, (n,) * 3)
    bv = O.to_dense(B).ravel()
    xv = np.linalg.solve(A, bv)
    lv = np.linalg.solve(A.T, xv - O.to_dense(Xt).ravel())
    UB = np.kron(np.kron(B.U[0], B.U[1]), B.U[2])
    assert np.linalg.norm(gb.ravel() - UB.T @ lv) <= 1e-7 * np.linalg.norm(UB.T @ lv)
    for j, (a, As) in enumerate(terms):
        dAj = O.dense_operator([(1.0, As)], (n,) * 3)
        assert abs(ga[j] - (-lv @ (dAj @ xv))) <= 1e-7 * abs(ga[j])
    # central differences of forward solves (h relative 1e-5)
    def f(al, bc):
        return float(_loss(tk, torch.tensor(al, dtype=torch.float64, device="cuda"),
                           torch.tensor(bc, dtype=torch.float64, device="cuda"), problem))
    for j in range(3):
        h = 1e-5 * theta[j]
        ap, am = list(theta), list(theta)
        ap[j] += h
        am[j] -= h
        fd = (f(ap, B.core) - f(am, B.core)) / (2 * h)
        assert abs(fd - ga[j]) <= 1e-4 * abs(ga[j]), (j, fd, ga[j])
    idx = (0, 1, 1)
    h = 1e-5 * abs(B.core[idx])
    cp, cm = B.core.copy(), B.core.copy()
    cp[idx] += h
    cm[idx] -= h
    fd = (f(theta, cp) - f(theta, cm)) / (2 * h)
    assert abs(fd - gb[idx]) <= 1e-4 * abs(gb[idx]), (fd, gb[idx])


def test_autograd_unconverged_solve_raises(tk):
    terms, theta, B, Xt, S, Om, oprm, problem = _problem(tk, 10, maxiter=2, max_restarts=1)
    alpha = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
    b_core = torch.tensor(B.core, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="forward solve ended with status"):
        _loss(tk, alpha, b_core, problem)
