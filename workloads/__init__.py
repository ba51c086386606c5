"""Seeded synthetic workloads for the Tucker-sketched GMRES hot path.

This module only *draws and assembles inputs*: Kronecker-sum operator factors,
right-hand sides in Tucker format, and the Gaussian sketch matrices that both
the CPU oracle and the GPU library consume.  It contains none of the solver's
arithmetic (no operator application, RoundSum, sketching or least squares), so
the oracle and the HIP path can share it without sharing the method.

Random streams
--------------
* ``numpy.random.default_rng(0)`` draws the sketches, in this order:
  S_1..S_d (n_k x s, the Khatri-Rao sGMRES sketch of Alg. 2) and then
  Omega_1..Omega_d (n_k x (cap + p), the pool of RoundSum range-finder test
  matrices of Sec. 3.1; every RoundSum uses the leading s_r columns).
  Entries are N(0, 1), unscaled.
* ``numpy.random.default_rng(1)`` draws the problem data (RHS cores/factors,
  noise, perturbation matrices, diffusion coefficients).

Operators are lists of terms ``(alpha, [A_1, ..., A_d])`` meaning
``L(X) = sum_j alpha_j X x_1 A_j^(1) ... x_d A_j^(d)`` (Eq. (2) of the paper,
read mode-wise); ``None`` stands for the identity.  Matrices are dense
row-major ``float64`` arrays.

Workloads (sizes of the five benchmark configurations):
  1  3D Poisson, n=32, all-ones rank-1 RHS, cap 10            (Sec. 3.4 Laplacian)
  2  3D convection-diffusion, n=256, 6 Kronecker terms, cap 32 (Sec. 4.2)
  3  3D Tikhonov-regularised deblurring, n=512, cap 48        (Sec. 4.3)
  4  3D Poisson with per-mode coefficients theta_k, n=256      (adjoint workload)
  5  4D Poisson + rank-2 Kronecker perturbation, n=128, cap 32
Every configuration accepts overrides of ``n`` and ``cap`` so tests can build
small copies with the same structure.
"""
from __future__ import annotations

import dataclasses
import hashlib
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Workload", "make_config", "laplacian_1d", "centered_difference_1d",
    "gaussian_blur_toeplitz", "draw_sketches", "CONFIG_DEFAULTS",
]


@dataclasses.dataclass
class Workload:
    """All inputs of one solve.  Arrays are float64, factors column-major
    (``U[k]`` has shape (n_k, r_k)), cores C-ordered (mode d fastest)."""
    name: str
    d: int
    n: List[int]
    terms: List[Tuple[float, List[Optional[np.ndarray]]]]
    b_core: np.ndarray
    b_factors: List[np.ndarray]
    S: List[np.ndarray]          # sGMRES Khatri-Rao sketch factors, n_k x s
    Omega: List[np.ndarray]      # RoundSum range-finder pool, n_k x (cap + p)
    cap: int
    p: int
    s: int
    k_trunc: int
    maxiter: int
    tol: float
    eta: float
    extra: dict = dataclasses.field(default_factory=dict)


CONFIG_DEFAULTS = {
    1: dict(d=3, n=32, cap=10, k_trunc=2),
    2: dict(d=3, n=256, cap=32, k_trunc=2),
    3: dict(d=3, n=512, cap=48, k_trunc=2),
    4: dict(d=3, n=256, cap=32, k_trunc=2),
    5: dict(d=4, n=128, cap=32, k_trunc=3),
}


def laplacian_1d(n: int) -> np.ndarray:
    """(n+1)^2 * tridiag(-1, 2, -1), the n x n second-difference matrix on the
    interior of a unit interval with step h = 1/(n+1) (Sec. 3.4, Laplacian)."""
    L = np.zeros((n, n))
    i = np.arange(n)
    L[i, i] = 2.0
    L[i[:-1], i[:-1] + 1] = -1.0
    L[i[1:], i[1:] - 1] = -1.0
    return L * float(n + 1) ** 2


def laplacian_eigenpairs(n: Sequence[int]):
    """Eigenpairs of ``laplacian_1d(n_k)`` for every mode in closed form (the
    DST-I basis): ``V[i, j] = sqrt(2/(n+1)) sin((i+1)(j+1) pi/(n+1))`` and
    ``lambda_j = 4 (n+1)^2 sin^2((j+1) pi/(2(n+1)))``.  Input data of the
    exponential-sum preconditioner of Sec. 3.4 on the GPU path; returns
    ``([V_k], [lambda_k])`` as NumPy arrays."""
    Vs, lams = [], []
    for nk in n:
        i = np.arange(1, nk + 1)
        Vs.append(np.sqrt(2.0 / (nk + 1)) * np.sin(np.outer(i, i) * np.pi / (nk + 1)))
        lams.append(4.0 * (nk + 1) ** 2 * np.sin(i * np.pi / (2 * (nk + 1))) ** 2)
    return Vs, lams


def centered_difference_1d(n: int) -> np.ndarray:
    """(n+1)/2 * tridiag(-1, 0, +1): centred first difference, sub-diagonal
    -1 and super-diagonal +1."""
    D = np.zeros((n, n))
    i = np.arange(n - 1)
    D[i, i + 1] = 1.0
    D[i + 1, i] = -1.0
    return D * (float(n + 1) / 2.0)


def gaussian_blur_toeplitz(n: int, sigma: float = 3.0, halfwidth: int = 12) -> np.ndarray:
    """Symmetric banded Toeplitz Gaussian blur: taps exp(-t^2/(2 sigma^2)) for
    |t| <= halfwidth, normalised so the full stencil sums to one; zero
    boundary (rows near the edge therefore sum to less than one)."""
    t = np.arange(-halfwidth, halfwidth + 1, dtype=np.float64)
    w = np.exp(-t * t / (2.0 * sigma * sigma))
    w /= w.sum()
    K = np.zeros((n, n))
    for off, wt in zip(range(-halfwidth, halfwidth + 1), w):
        if abs(off) >= n:
            continue
        idx = np.arange(max(0, -off), min(n, n - off))
        K[idx, idx + off] = wt
    return K


def noisy_blur_problem(n: int, seed: int = 5, noise: float = 0.05, sigma: float = 1.5, halfwidth: int = 6,
                       rank: int = 2):
    """Small ill-posed deblurring problem for the regularised solves: K the
    Gaussian blur (``gaussian_blur_toeplitz``), X_true a rank-(rank,)*3 Tucker
    image with N(0,1) core and factors, Y = X_true x_k K plus white noise of
    relative level ``noise`` (dense, n^3).  Returns (K, Y, (core, factors) of
    X_true, rng) with the rng positioned after the draws."""
    rng = np.random.default_rng(seed)
    K = gaussian_blur_toeplitz(n, sigma=sigma, halfwidth=halfwidth)
    Xc = rng.standard_normal((rank,) * 3)
    XU = [rng.standard_normal((n, rank)) for _ in range(3)]
    KU = [K @ u for u in XU]
    Y = np.einsum("abc,ia,jb,kc->ijk", Xc, KU[0], KU[1], KU[2])
    Y = Y + noise * np.linalg.norm(Y) / np.sqrt(Y.size) * rng.standard_normal(Y.shape)
    return K, Y, (Xc, XU), rng


def hollow_bars(n: int, nbars: int, rng):
    """Tucker form of a phantom of ``nbars`` hollow axis-aligned bars (a
    stand-in with the structure of the inverse-problem experiment's phantom):
    each bar is an outer box minus an inner box, two rank-1 indicator tensors,
    so the factors hold 2 * nbars indicator vectors per mode and the core is
    superdiagonal with entries +1 (outer) and -1 (inner)."""
    r = 2 * nbars
    U = [np.zeros((n, r)) for _ in range(3)]
    core = np.zeros((r,) * 3)
    for b in range(nbars):
        for k in range(3):
            lo = int(rng.integers(n // 8, n // 2))
            hi = int(rng.integers(lo + n // 4, min(n - n // 16, lo + 3 * n // 4)))
            wall = max(2, (hi - lo) // 5)
            U[k][lo:hi, 2 * b] = 1.0
            U[k][lo + wall:hi - wall, 2 * b + 1] = 1.0
        core[2 * b, 2 * b, 2 * b] = 1.0
        core[2 * b + 1, 2 * b + 1, 2 * b + 1] = -1.0
    return core, U


def deblur_gcv_problem(n: int = 256, nbars: int = 3, rank_b: int = 32, noise: float = 0.05,
                       sigma: float = 3.0, halfwidth: int = 12, seed: int = 3):
    """Regularised deblurring workload (the setting of the inverse-problem
    experiment: blur operator K (x) K (x) K, noisy data compressed to Tucker
    format before the solve).  X_true: ``hollow_bars`` phantom; Y = X_true x_k K
    plus white noise of relative level ``noise``; B = truncated HOSVD of Y to
    rank (rank_b,)*3.  Returns (K, (B core, B factors), (X_true core,
    factors)); cached on disk by its parameters."""
    K = gaussian_blur_toeplitz(n, sigma=sigma, halfwidth=halfwidth)
    key = f"deblur-gcv-v2-n{n}-b{nbars}-rb{rank_b}-e{noise}-s{sigma}-h{halfwidth}-seed{seed}"
    path = _cache_path(key)
    rng = np.random.default_rng(seed)
    Xc, XU = hollow_bars(n, nbars, rng)
    if os.path.exists(path):
        z = np.load(path)
        return K, (z["core"], [z["Q0"], z["Q1"], z["Q2"]]), (Xc, XU)
    KU = [K @ U for U in XU]
    Y = np.einsum("abc,ia,jb,kc->ijk", Xc, KU[0], KU[1], KU[2], optimize=True)
    scale = noise * np.linalg.norm(Y) / np.sqrt(Y.size)
    Y += scale * rng.standard_normal(Y.shape)
    core, Q = _hosvd_truncate_dense(Y, [rank_b] * 3)
    del Y
    np.savez(path, core=core, Q0=Q[0], Q1=Q[1], Q2=Q[2])
    return K, (core, Q), (Xc, XU)


def draw_sketches(n: Sequence[int], s: int, cap: int, p: int, seed: int = 0):
    """Gaussian N(0,1) sketches from one seeded stream: S_1..S_d (n_k x s)
    then Omega_1..Omega_d (n_k x (cap+p))."""
    rng = np.random.default_rng(seed)
    S = [rng.standard_normal((nk, s)) for nk in n]
    Om = [rng.standard_normal((nk, cap + p)) for nk in n]
    return S, Om


def draw_mln_sketches(n: Sequence[int], r: int, p: int, seed: int = 7):
    """Gaussian N(0,1) multilinear Nystrom sketches Psi_1..Psi_d
    (n_k x (r + p)) from one seeded stream."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((nk, r + p)) for nk in n]


def _gaussian_tucker(rng, n, ranks):
    core = rng.standard_normal(tuple(ranks))
    U = [rng.standard_normal((nk, rk)) for nk, rk in zip(n, ranks)]
    return core, U


def _hosvd_truncate_dense(Y: np.ndarray, ranks):
    """Truncated HOSVD of a dense tensor (input preparation only): leading
    left singular vectors of each unfolding, core = Y x_k Q_k^T."""
    d = Y.ndim
    Q = []
    for k in range(d):
        Yk = np.moveaxis(Y, k, 0).reshape(Y.shape[k], -1)
        Gk = Yk @ Yk.T
        w, V = np.linalg.eigh(Gk)
        Q.append(V[:, ::-1][:, : ranks[k]].copy())
    core = Y
    for k in range(d):
        core = np.moveaxis(np.tensordot(Q[k].T, core, axes=([1], [k])), 0, k)
    return np.ascontiguousarray(core), Q


def _cache_path(key: str) -> str:
    base = os.environ.get("TSGMRES_CACHE", "/tmp/tsgmres_workloads")
    os.makedirs(base, exist_ok=True)
    return os.path.join(base, hashlib.sha1(key.encode()).hexdigest()[:16] + ".npz")


def _deblur_rhs(n: int, rank: int, noise_var: float, rng, K: np.ndarray):
    """RHS of the deblurring workload: Y = X_true x_k K + noise (dense, iid
    N(0, noise_var)), compressed by truncated HOSVD to (rank,)*3, then
    B = Y_c x_k K^T (normal equations right-hand side)."""
    key = f"deblur-v1-n{n}-r{rank}-v{noise_var}"
    path = _cache_path(key)
    if os.path.exists(path):
        z = np.load(path)
        return z["core"], [z["Q0"], z["Q1"], z["Q2"]], z["Xc"], [z["XU0"], z["XU1"], z["XU2"]]
    Xc, XU = _gaussian_tucker(rng, [n] * 3, [rank] * 3)
    # blurred signal, dense
    KU = [K @ U for U in XU]
    Y = np.einsum("abc,ia,jb,kc->ijk", Xc, KU[0], KU[1], KU[2], optimize=True)
    Y += np.sqrt(noise_var) * rng.standard_normal(Y.shape)
    core, Q = _hosvd_truncate_dense(Y, [rank] * 3)
    del Y
    np.savez(path, core=core, Q0=Q[0], Q1=Q[1], Q2=Q[2], Xc=Xc, XU0=XU[0], XU1=XU[1], XU2=XU[2])
    return core, Q, Xc, XU


def make_config(cfg: int, n: Optional[int] = None, cap: Optional[int] = None,
                p: int = 5, maxiter: int = 60, s: Optional[int] = None,
                tol: float = 1e-8, eta: float = 0.4,
                k_trunc: Optional[int] = None) -> Workload:
    """Build workload ``cfg`` (1..5).  ``n``/``cap`` override the sizes of the
    full configuration while keeping its structure and seeds."""
    if cfg not in CONFIG_DEFAULTS:
        raise ValueError(f"unknown workload {cfg}")
    dflt = CONFIG_DEFAULTS[cfg]
    d = dflt["d"]
    n = int(n if n is not None else dflt["n"])
    cap = int(cap if cap is not None else dflt["cap"])
    k_trunc = int(k_trunc if k_trunc is not None else dflt["k_trunc"])
    s = int(s if s is not None else 2 * maxiter)
    ns = [n] * d
    rng = np.random.default_rng(1)
    extra = {}
    eye = None
    if cfg == 1:
        L = laplacian_1d(n)
        terms = [(1.0, [L if j == k else eye for j in range(d)]) for k in range(d)]
        b_core = np.ones((1,) * d)
        b_U = [np.ones((n, 1)) for _ in range(d)]
        name = f"poisson3d_n{n}"
    elif cfg == 2:
        eps, c = 1e-2, [1.0, 0.5, 0.25]
        L = laplacian_1d(n)
        D = centered_difference_1d(n)
        terms = []
        for k in range(d):
            terms.append((eps, [L if j == k else eye for j in range(d)]))
        for k in range(d):
            terms.append((c[k], [D if j == k else eye for j in range(d)]))
        b_core, b_U = _gaussian_tucker(rng, ns, [3] * d)
        name = f"convdiff3d_n{n}"
    elif cfg == 3:
        lam = 1e-3
        K = gaussian_blur_toeplitz(n)
        M = K.T @ K
        terms = [(1.0, [M, M, M]), (lam, [eye, eye, eye])]
        core, Q, Xc, XU = _deblur_rhs(n, 5, 1e-4, rng, K)
        b_core = core
        b_U = [K.T @ q for q in Q]
        extra.update(K=K, lam=lam, x_true_core=Xc, x_true_factors=XU)
        name = f"deblur3d_n{n}"
    elif cfg == 4:
        theta = rng.uniform(0.5, 2.0, size=d)
        L = laplacian_1d(n)
        terms = [(float(theta[k]), [L if j == k else eye for j in range(d)]) for k in range(d)]
        b_core = np.ones((1,) * d)
        b_U = [np.ones((n, 1)) for _ in range(d)]
        xt_core, xt_U = _gaussian_tucker(rng, ns, [4] * d)
        extra.update(theta=theta, L=L, x_target_core=xt_core, x_target_factors=xt_U)
        name = f"poisson3d_theta_n{n}"
    elif cfg == 5:
        L = laplacian_1d(n)
        terms = [(1.0, [L if j == k else eye for j in range(d)]) for k in range(d)]
        for _ in range(2):
            Rs = [rng.standard_normal((n, n)) / np.sqrt(n) for _ in range(d)]
            terms.append((1.0, [np.eye(n) + 0.01 * R for R in Rs]))
        b_core, b_U = _gaussian_tucker(rng, ns, [4] * d)
        name = f"poisson4d_pert_n{n}"
    S, Om = draw_sketches(ns, s, cap, p, seed=0)
    return Workload(name=name, d=d, n=ns, terms=terms, b_core=np.ascontiguousarray(b_core),
                    b_factors=[np.asarray(u, dtype=np.float64) for u in b_U], S=S, Omega=Om,
                    cap=cap, p=p, s=s, k_trunc=k_trunc, maxiter=maxiter, tol=tol, eta=eta,
                    extra=extra)
