"""RoundSum: randomized RHOSVD recompression of a sum of Tucker tensors
(Sec. 3.1) -- oracle, test infrastructure only.

Steps, in the paper's order:
  1. effective-rank heuristic on the energy-weighted concatenated factors
     ``V_k = [||G^(1)|| U_k^(1), ..., ||G^(N)|| U_k^(N)]`` (eigenvalues of
     their Gram matrix) -> uniform sketch width ``s = max_k r~_k + p``;
  2. Khatri-Rao range sketch ``Y_k = sum_i U_k^(i) G_(k)^(i) (KRP_{j!=k} M_j^(i))``
     with ``M_j^(i) = U_j^(i)T S_j``;
  3. economy (Householder) QR of Y_k -> orthonormal U^_k;
  4. core projection ``C^ = sum_i G^(i) x_k (U^_k^T U_k^(i))``;
  5. ST-HOSVD of C^ to the tolerance eps.

Readings where the paper leaves a choice:
  * weights are |c_i| ||G^(i)||_F (the coefficient of a summand scales its
    energy); the Gram is formed on the smaller side (R_k x R_k or n_k x n_k),
    at every size: both sides have the same nonzero eigenvalues;
  * eigenvalues below ``delta * lambda_max`` (delta = 1e-12, ~30x above the
    rounding level of a 512-wide FP64 Gram) are treated as zero, then
    ``r~_k = min{r : sum_{i>r} lambda_i <= tau^2 sum_i lambda_i}``;
  * ``s = min(max_k r~_k + p, cap + p)``; the range-finder test matrices are
    the leading s columns of a fixed pool Omega_k drawn once, and mode k keeps
    ``min(s, n_k)`` orthonormal columns from its QR;
  * ST-HOSVD visits modes 1..d, uses a true SVD of each unfolding, keeps
    ``r_k = min{r >= 1 : sum_{i>r} sigma_i^2 <= eps^2 ||C^||^2 / d}``
    capped at ``cap`` (or the forced rank, for rank replay);
  * a sum whose projected core has ||C^||_F <= 16 u sum_b |c_b| ||G^(b)||_F
    (u = 2^-53) is numerically zero -- below that level every digit of the
    result is rounding noise -- and returns a rank-(1,..,1) zero tensor.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence

import numpy as np

from .tucker import Tucker, multi_ttm, ttm, unfold

DELTA_CLAMP = 1e-12
ZERO_TOL = 16.0 * 2.0 ** -53


@dataclasses.dataclass
class RoundParams:
    eps: float = 1e-10              # ST-HOSVD relative tolerance
    cap: int = 48                   # rank cap per mode
    p: int = 5                      # oversampling of the range sketch
    tau: Optional[float] = None     # effective-rank threshold (default: eps)
    force_s: Optional[int] = None   # replay the sketch width
    force_ranks: Optional[Sequence[int]] = None   # replay output ranks
    delta: float = DELTA_CLAMP
    # step 3's orthonormal basis of range(Y_k): None = Householder QR.  Sec.
    # 3.1 fixes the range, not the basis; tests pass another valid basis
    # routine to measure how far that choice alone moves a trajectory.
    range_basis: Optional[Callable[[np.ndarray], np.ndarray]] = None
    # rounding applied to every summand's core and factors on entry (None:
    # none); tests pass a round-to-FP32 map to model a reduced-precision form
    operand_rounding: Optional[Callable[[np.ndarray], np.ndarray]] = None


def _rank_from_tail(vals_desc: np.ndarray, thresh: float) -> int:
    """min{r >= 0 : sum_{i>r} v_i <= thresh} for a descending nonnegative array."""
    tail = np.concatenate([np.cumsum(vals_desc[::-1])[::-1], [0.0]])   # tail[r] = sum_{i>=r}
    ok = np.nonzero(tail <= thresh)[0]
    return int(ok[0])


def effective_sketch_size(blocks, prm: RoundParams):
    """Step 1 (Sec. 3.1): per-mode effective rank of the energy-weighted
    concatenated factors, then the uniform sketch width.  Returns
    ``(s, [r~_k])``."""
    d = blocks[0][1].d
    n = blocks[0][1].n
    tau = prm.eps if prm.tau is None else prm.tau
    w = [abs(c) * np.linalg.norm(X.core.ravel()) for c, X in blocks]
    rt = []
    for k in range(d):
        V = np.concatenate([wb * X.U[k] for wb, (_, X) in zip(w, blocks)], axis=1)
        R = V.shape[1]
        Gm = V.T @ V if R <= n[k] else V @ V.T
        lam = np.sort(np.linalg.eigvalsh(Gm))[::-1]
        if lam.size == 0 or lam[0] <= 0.0:
            rt.append(0)
            continue
        lam = np.where(lam > prm.delta * lam[0], lam, 0.0)
        rt.append(_rank_from_tail(lam, tau * tau * lam.sum()))
    big = prm.cap + prm.p
    est = max(r + prm.p for r in rt)
    s = min(est, big)
    return int(s), rt


def st_hosvd(C: np.ndarray, eps: float, cap: int, force_ranks=None, zero: bool = False):
    """Sequentially truncated HOSVD of a small dense core (step 5): modes in
    order 1..d, thin SVD of the current unfolding, per-mode budget
    eps^2 ||C||^2 / d.  Returns (core, [V_k], ranks)."""
    d = C.ndim
    total = 0.0 if zero else float(np.sum(C * C))
    Vs, ranks = [], []
    for k in range(d):
        Ck = unfold(C, k)
        Us, sig, _ = np.linalg.svd(Ck, full_matrices=False)
        if force_ranks is not None:
            r = int(min(force_ranks[k], Us.shape[1]))
        elif total == 0.0:
            r = 1
        else:
            r = max(1, _rank_from_tail(sig * sig, eps * eps * total / d))
            r = min(r, cap)
        Vk = Us[:, :r]
        C = ttm(C, Vk.T, k)
        Vs.append(Vk)
        ranks.append(r)
    return C, Vs, ranks


def _mttkrp(G: np.ndarray, Ms: List[np.ndarray], k: int) -> np.ndarray:
    """MTTKRP (Def. MTTKRP) on a core: ``T[i_k, l] = sum_{i_j, j!=k} G[i]
    prod_{j!=k} M_j[i_j, l]`` -- the core unfolding times the Khatri-Rao
    product of the other modes' matrices (column-wise Kronecker)."""
    d = G.ndim
    s = Ms[(k + 1) % d].shape[1]
    out = np.zeros((G.shape[k], s))
    for l in range(s):
        T = G
        for j in range(d - 1, -1, -1):
            if j == k:
                continue
            T = np.tensordot(T, Ms[j][:, l], axes=([j], [0]))
        out[:, l] = T
    return out


def roundsum(blocks, Omega: Sequence[np.ndarray], prm: RoundParams):
    """RoundSum of Sec. 3.1 applied to ``sum_b c_b X_b``.  Returns
    ``(Tucker, info)`` with ``info = dict(s=..., ranks=..., rtilde=...)``."""
    d = blocks[0][1].d
    if prm.operand_rounding is not None:
        f = prm.operand_rounding
        blocks = [(c, Tucker(f(X.core), [f(u) for u in X.U])) for c, X in blocks]
    # 1. effective-rank heuristic -> sketch width
    s, rt = effective_sketch_size(blocks, prm)
    if prm.force_s is not None:
        s = int(prm.force_s)
    Om = [O[:, :s] for O in Omega]
    # 2. Khatri-Rao range sketch of every mode unfolding
    Y = [0.0] * d
    for c, X in blocks:
        M = [X.U[j].T @ Om[j] for j in range(d)]          # r_j x s
        for k in range(d):
            Y[k] = Y[k] + c * (X.U[k] @ _mttkrp(X.core, M, k))
    # 3. economy QR (Householder), or the given basis routine
    if prm.range_basis is None:
        Uh = [np.linalg.qr(Yk, mode="reduced")[0] for Yk in Y]
    else:
        Uh = [prm.range_basis(Yk) for Yk in Y]
    # 4. core projection
    C = None
    for c, X in blocks:
        T = c * multi_ttm(X.core, [Uh[k].T @ X.U[k] for k in range(d)])
        C = T if C is None else C + T
    # 5. ST-HOSVD of the projected core
    wsum = sum(abs(c) * np.linalg.norm(X.core.ravel()) for c, X in blocks)
    zero = float(np.linalg.norm(C.ravel())) <= ZERO_TOL * wsum
    core, Vs, ranks = st_hosvd(C, prm.eps, prm.cap, prm.force_ranks, zero=zero)
    U = [Uh[k] @ Vs[k] for k in range(d)]
    if zero and prm.force_ranks is None:
        core = np.zeros((1,) * d)
        U = [np.eye(u.shape[0], 1) for u in U]
        ranks = [1] * d
    return Tucker(np.ascontiguousarray(core), U), dict(s=s, ranks=ranks, rtilde=rt)
