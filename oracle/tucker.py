"""Tucker-format primitives of the oracle (test infrastructure only).

Conventions: a Tucker tensor is ``X = G x_1 U_1 ... x_d U_d`` (Sec. 2.3,
Tucker format equation) with a C-ordered core ``G`` of shape (r_1..r_d) and
factors ``U_k`` of shape (n_k, r_k).  ``vec`` is row-major (mode d fastest),
under which ``X x_1 A_1 ... x_d A_d`` has ``vec = (A_1 kron ... kron A_d) vec(X)``.
A *block sum* is a list of ``(coef, Tucker)`` pairs meaning ``sum coef * X``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Tucker:
    core: np.ndarray
    U: List[np.ndarray]

    @property
    def d(self) -> int:
        return self.core.ndim

    @property
    def ranks(self) -> Tuple[int, ...]:
        return tuple(self.core.shape)

    @property
    def n(self) -> Tuple[int, ...]:
        return tuple(u.shape[0] for u in self.U)


def ttm(T: np.ndarray, M: np.ndarray, k: int) -> np.ndarray:
    """Mode-k tensor-times-matrix ``T x_k M`` (Def. TTM, Sec. 2.2):
    ``Y_(k) = M T_(k)``, i.e. every mode-k fibre is multiplied by M."""
    Y = np.tensordot(M, T, axes=([1], [k]))
    return np.moveaxis(Y, 0, k)


def multi_ttm(T: np.ndarray, Ms: Sequence[Optional[np.ndarray]]) -> np.ndarray:
    """``T x_1 M_1 ... x_d M_d``; ``None`` skips a mode."""
    for k, M in enumerate(Ms):
        if M is not None:
            T = ttm(T, M, k)
    return T


def unfold(T: np.ndarray, k: int) -> np.ndarray:
    """Mode-k unfolding: rows indexed by i_k, columns by the other indices
    in their natural (row-major) order."""
    return np.moveaxis(T, k, 0).reshape(T.shape[k], -1)


def to_dense(X: Tucker) -> np.ndarray:
    """Full tensor of a Tucker tensor (tiny sizes only)."""
    return multi_ttm(X.core, X.U)


def block_dense(blocks) -> np.ndarray:
    return sum(c * to_dense(X) for c, X in blocks)


def scale(X: Tucker, a: float) -> Tucker:
    return Tucker(X.core * a, [u.copy() for u in X.U])


def transpose_terms(terms):
    """Terms of the adjoint operator: every factor transposed."""
    return [(a, [None if A is None else A.T.copy() for A in As]) for a, As in terms]


def dense_operator(terms, n: Sequence[int]) -> np.ndarray:
    """Dense matrix ``sum_j alpha_j A_j^(1) kron ... kron A_j^(d)`` of Eq. (2)
    under row-major vec (tiny grids only)."""
    N = int(np.prod(n))
    Ld = np.zeros((N, N))
    for a, As in terms:
        K = np.ones((1, 1))
        for k, A in enumerate(As):
            K = np.kron(K, np.eye(n[k]) if A is None else A)
        Ld += a * K
    return Ld


def apply_op(terms, X: Tucker, transpose: bool = False):
    """Kronecker-sum operator applied to a Tucker tensor (Eq. (2), step 'L(W)'
    of Alg. 2): term j contributes ``alpha_j * G x_k (A_j^(k) U_k)``, all
    terms sharing the core G; identity factors leave U_k untouched.
    Returns the (unrounded) block sum."""
    blocks = []
    for a, As in terms:
        U = []
        for k, A in enumerate(As):
            if A is None:
                U.append(X.U[k])
            else:
                U.append((A.T if transpose else A) @ X.U[k])
        blocks.append((float(a), Tucker(X.core, U)))
    return blocks


def sketch_krp(blocks, S: Sequence[np.ndarray]) -> np.ndarray:
    """Khatri-Rao sketch ``S^T vec(X)`` with ``S = S_1 (.) ... (.) S_d``
    (Alg. 2, lines building b_s and the columns of M).  Column l of the
    Khatri-Rao product is ``S_1[:,l] kron ... kron S_d[:,l]`` (Def. KRP), so
    ``(S^T vec X)_l = X x_1 S_1[:,l]^T ... x_d S_d[:,l]^T``; for a Tucker
    term this is ``sum_i G[i] prod_k P_k[l, i_k]`` with ``P_k = S_k^T U_k``."""
    s = S[0].shape[1]
    out = np.zeros(s)
    for c, X in blocks:
        P = [Sk.T @ Uk for Sk, Uk in zip(S, X.U)]          # s x r_k
        for l in range(s):
            T = X.core
            for k in range(X.d - 1, -1, -1):   # contract the last remaining mode
                T = T @ P[k][l]
            out[l] += c * float(T)
    return out


def sketch_kron(blocks, S: Sequence[np.ndarray]) -> np.ndarray:
    """Full Kronecker sketch ``X x_1 S_1^T ... x_d S_d^T`` (an s^d core); its
    superdiagonal equals the Khatri-Rao sketch (Sec. 3.3, diag identity)."""
    out = None
    for c, X in blocks:
        P = [Sk.T @ Uk for Sk, Uk in zip(S, X.U)]
        T = c * multi_ttm(X.core, P)
        out = T if out is None else out + T
    return out


def inner(X: Tucker, Y: Tucker) -> float:
    """Frobenius inner product ``<X, Y>`` (Alg. 2, orthogonalisation
    coefficients): ``<G_X, G_Y x_1 (U_1^X)^T U_1^Y ... >``."""
    Ms = [ux.T @ uy for ux, uy in zip(X.U, Y.U)]
    return float(np.sum(X.core * multi_ttm(Y.core, Ms)))


def exact_norm(blocks) -> float:
    """Frobenius norm of a block sum without cancellation: per mode, a
    Householder QR of the concatenated factors ``[U_k^(1), ..., U_k^(T)] =
    Q_k R_k``; then ``||sum_b c_b G_b x_k R_k[:, cols_b]||_F``.  (The sum of
    pairwise inner products is not used: it loses all digits below
    sqrt(eps) of the largest term.)"""
    d = blocks[0][1].d
    Rs = []
    for k in range(d):
        Ucat = np.concatenate([X.U[k] for _, X in blocks], axis=1)
        _, R = np.linalg.qr(Ucat, mode="reduced")
        Rs.append(R)
    core = None
    offs = [0] * d
    for c, X in blocks:
        sl = []
        for k in range(d):
            r = X.U[k].shape[1]
            sl.append(Rs[k][:, offs[k]:offs[k] + r])
            offs[k] += r
        T = c * multi_ttm(X.core, sl)
        core = T if core is None else core + T
    return float(np.linalg.norm(core.ravel()))
