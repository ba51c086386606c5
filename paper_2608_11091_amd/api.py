"""Torch-facing wrappers of the C ABI (argument marshalling only).

Every numerical step runs in the HIP library; this module only lays out
device buffers with PyTorch, fills the ABI structs and reads results back.

Layouts (see ``include/tsgmres.h``):
  * ``Tucker.core``: float64 CUDA tensor of shape ``rcap`` (C order);
  * ``Tucker.U[k]``: float64 CUDA tensor of shape ``(rcap_k, n_k)`` -- the
    row-major view of a column-major ``n_k x rcap_k`` factor;
  * operator factors: ``(n_k, n_k)`` row-major tensors or ``None``;
  * sketch factors ``S_k``: ``(s, n_k)`` (column-major ``n_k x s``) and
    ``Omega_k``: ``(cap + p, n_k)``;
  * multilinear Nystrom sketches ``Psi_k``: ``(r + p, n_k)``; factor
    sketches ``F_k``: ``(r, n_k)`` (column-major ``n_k x r``); sketched core:
    ``(r + p,) * d`` (C order).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _abi
from ._abi import (TK_MAX_D, TkBlockSum, TkKronOp, TkMlnParams, TkRoundParams, TkSgmresInfo, TkSgmresParams,
                   TkTucker, check)

__all__ = ["Tucker", "KronOp", "SolveParams", "apply_op", "sketch", "rhosvd", "norm", "solve", "backward",
           "TuckerSGMRESLoss", "storage_floats", "kernel_timer", "kernel_timer_read", "solve_workspace_bytes",
           "MlnParams", "mln_sketch", "mln_recover", "mln_solve", "mln_solve_workspace_bytes",
           "precond_tensors", "project_core"]


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


@dataclasses.dataclass
class Tucker:
    """Tucker tensor on the GPU with capacity-padded core and factors."""
    core: torch.Tensor
    U: List[torch.Tensor]
    ranks: Tuple[int, ...]

    @property
    def d(self) -> int:
        return self.core.dim()

    @property
    def n(self) -> Tuple[int, ...]:
        return tuple(int(u.shape[1]) for u in self.U)

    @property
    def rcap(self) -> Tuple[int, ...]:
        return tuple(int(s) for s in self.core.shape)

    @staticmethod
    def empty(n: Sequence[int], rcap: Sequence[int], device="cuda") -> "Tucker":
        core = torch.zeros(tuple(rcap), dtype=torch.float64, device=device)
        U = [torch.zeros((r, nk), dtype=torch.float64, device=device) for nk, r in zip(n, rcap)]
        return Tucker(core, U, tuple(1 for _ in n))

    @staticmethod
    def from_numpy(core: np.ndarray, factors: Sequence[np.ndarray], device="cuda",
                   rcap: Optional[Sequence[int]] = None) -> "Tucker":
        ranks = tuple(core.shape)
        rcap = tuple(rcap) if rcap is not None else ranks
        c = np.zeros(rcap)
        c[tuple(slice(0, r) for r in ranks)] = core
        Us = []
        for k, u in enumerate(factors):
            ut = np.zeros((rcap[k], u.shape[0]))
            ut[: u.shape[1]] = u.T
            Us.append(torch.from_numpy(ut).to(device))
        return Tucker(torch.from_numpy(c).to(device), Us, ranks)

    def to_numpy(self):
        r = self.ranks
        core = self.core[tuple(slice(0, x) for x in r)].cpu().numpy().copy()
        U = [self.U[k][: r[k]].cpu().numpy().T.copy() for k in range(self.d)]
        return core, U

    def struct(self) -> TkTucker:
        t = TkTucker()
        t.d = self.d
        for k in range(self.d):
            t.n[k] = self.n[k]
            t.r[k] = self.ranks[k]
            t.rcap[k] = self.rcap[k]
            t.U[k] = _ptr(self.U[k])
        t.core = _ptr(self.core)
        return t


def _blocks_struct(blocks: Sequence[Tuple[float, Tucker]]):
    arr = (TkTucker * len(blocks))(*[b.struct() for _, b in blocks])
    coef = (C.c_double * len(blocks))(*[float(c) for c, _ in blocks])
    bs = TkBlockSum()
    bs.nblocks = len(blocks)
    bs.coef = coef
    bs.blocks = arr
    return bs, (arr, coef)


@dataclasses.dataclass
class KronOp:
    """``L(X) = sum_j alpha_j X x_1 A_j^(1) ... x_d A_j^(d)`` (row-major factors)."""
    alpha: List[float]
    A: List[List[Optional[torch.Tensor]]]

    @property
    def d(self) -> int:
        return len(self.A[0])

    @property
    def nterms(self) -> int:
        return len(self.alpha)

    @staticmethod
    def from_terms(terms, device="cuda") -> "KronOp":
        cache = {}

        def dev(A):
            if A is None:
                return None
            key = id(A)
            if key not in cache:
                cache[key] = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float64)).to(device)
            return cache[key]
        return KronOp([float(a) for a, _ in terms], [[dev(A) for A in As] for _, As in terms])

    def struct(self, n: Sequence[int]):
        op = TkKronOp()
        op.d = self.d
        for k in range(self.d):
            op.n[k] = n[k]
        op.nterms = self.nterms
        alpha = (C.c_double * self.nterms)(*self.alpha)
        ptrs = (C.c_void_p * (self.nterms * self.d))(*[_ptr(A) for As in self.A for A in As])
        op.alpha = alpha
        op.A = ptrs
        return op, (alpha, ptrs)


def _ptr_array(ts: Sequence[Optional[torch.Tensor]]):
    return (C.c_void_p * len(ts))(*[_ptr(t) for t in ts])


def apply_op(op: KronOp, x: Tucker, transpose: bool = False, form: int = 0):
    """Factor products of ``L(x)``; returns the block list ``[(alpha_j, Tucker)]``.
    ``form`` 1 computes them in FP32, 2 with bfloat16 operands on the BF16
    matrix cores (FP32 accumulation); results are widened to FP64."""
    lib = _abi.load()
    d = x.d
    AU = []
    for As in op.A:
        AU.append([None if A is None else torch.zeros_like(x.U[k]) for k, A in enumerate(As)])
    ops, keep = op.struct(x.n)
    xs = x.struct()
    out = _ptr_array([t for row in AU for t in row])
    nb = C.c_size_t()
    check(lib.tucker_apply_op_workspace(C.byref(ops), C.byref(xs), int(form), C.byref(nb)))
    ws = _workspace(nb.value, x.core.device)
    check(lib.tucker_apply_op(C.byref(ops), C.byref(xs), int(transpose), int(form), out, C.c_void_p(ws.data_ptr()),
                              nb.value, _stream()))
    blocks = []
    for j, As in enumerate(op.A):
        U = [x.U[k] if A is None else AU[j][k] for k, A in enumerate(As)]
        blocks.append((op.alpha[j], Tucker(x.core, U, x.ranks)))
    return blocks


def sketch(blocks, S: Sequence[torch.Tensor], form: int = 0) -> torch.Tensor:
    """Khatri-Rao sketch ``S^T vec(sum_b c_b X_b)`` (length s); ``form`` 1
    computes it in FP32, 2 with bfloat16 factor products."""
    lib = _abi.load()
    bs, keep = _blocks_struct(blocks)
    s = int(S[0].shape[0])
    dev = blocks[0][1].core.device
    out = torch.zeros(s, dtype=torch.float64, device=dev)
    nb = C.c_size_t()
    check(lib.tucker_sketch_workspace(C.byref(bs), s, int(form), C.byref(nb)))
    ws = _workspace(nb.value, dev)
    check(lib.tucker_sketch(C.byref(bs), _ptr_array(S), s, int(form), C.c_void_p(out.data_ptr()),
                            C.c_void_p(ws.data_ptr()), nb.value, _stream()))
    return out


def sketch_noalloc(blocks, S: Sequence[torch.Tensor], out: torch.Tensor, form: int = 0) -> torch.Tensor:
    """The Khatri-Rao sketch through the allocation-free entry point: the
    library uses its static device scratch instead of a workspace; ``out``
    (float64, length s, on the blocks' device) is written in place."""
    lib = _abi.load()
    bs, keep = _blocks_struct(blocks)
    s = int(S[0].shape[0])
    if out.dtype != torch.float64 or out.numel() < s or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of length >= s")
    check(lib.tucker_sketch_noalloc(C.byref(bs), _ptr_array(S), s, int(form), C.c_void_p(out.data_ptr()),
                                    _stream()))
    return out


def rhosvd(blocks, omega: Sequence[torch.Tensor], eps: float, cap: int, p: int = 5, tau: float = -1.0,
           force_s: int = -1, force_ranks: Optional[Sequence[int]] = None, out_rcap: Optional[Sequence[int]] = None,
           form: int = 0):
    """RoundSum of a block sum; returns ``(Tucker, s)``.  ``form`` 1 runs it in
    the FP32 form's arithmetic (FP64 range-sketch QR), 2 in the FP32 form
    with bfloat16 factor products."""
    lib = _abi.load()
    bs, keep = _blocks_struct(blocks)
    x0 = blocks[0][1]
    prm = TkRoundParams()
    prm.eps, prm.tau, prm.rank_cap, prm.oversample, prm.force_s = eps, tau, cap, p, force_s
    prm.form = int(form)
    for k in range(TK_MAX_D):
        prm.force_ranks[k] = -1 if force_ranks is None or k >= len(force_ranks) else int(force_ranks[k])
    rc = tuple(out_rcap) if out_rcap is not None else (cap,) * x0.d
    out = Tucker.empty(x0.n, rc, x0.core.device)
    os_ = out.struct()
    nb = C.c_size_t()
    check(lib.tucker_rhosvd_workspace(C.byref(bs), C.byref(prm), C.byref(nb)))
    ws = _workspace(nb.value, x0.core.device)
    s_out = C.c_int32(0)
    check(lib.tucker_rhosvd(C.byref(bs), C.byref(prm), _ptr_array(omega), C.byref(os_), C.byref(s_out),
                            C.c_void_p(ws.data_ptr()), nb.value, _stream()))
    out.ranks = tuple(int(os_.r[k]) for k in range(x0.d))
    return out, int(s_out.value)


def norm(blocks) -> float:
    """Exact Frobenius norm of a block sum (QR of concatenated factors)."""
    lib = _abi.load()
    bs, keep = _blocks_struct(blocks)
    dev = blocks[0][1].core.device
    nb = C.c_size_t()
    check(lib.tucker_norm_workspace(C.byref(bs), C.byref(nb)))
    ws = _workspace(nb.value, dev)
    out = C.c_double(0.0)
    check(lib.tucker_norm(C.byref(bs), C.byref(out), C.c_void_p(ws.data_ptr()), nb.value, _stream()))
    return float(out.value)


@dataclasses.dataclass
class SolveParams:
    form: int = 0            # 0 FP64, 1 FP32 cycles
    tol: float = 1e-8
    eta: float = 0.4
    maxiter: int = 60
    max_restarts: int = 50
    k_trunc: int = 2
    rank_cap: int = 48
    oversample: int = 5
    eps_trunc: float = -1.0
    eps_min: float = -1.0
    tol_inner_floor: float = -1.0
    # exponential-sum preconditioner (Sec. 3.4): q and the per-mode eigenpairs
    # (lists of device tensors: V_k as (n_k, n_k) holding the column-major
    # matrix, lambda_k of length n_k), e.g. ``precond_tensors(*workloads.laplacian_eigenpairs(n))``
    precond_q: int = 0
    precond: Optional[Tuple[list, list]] = None
    # projected Tikhonov with GCV on the sketched least squares (Sec. 4.3)
    tikhonov: bool = False
    # 0: RHOSVD-Tucker sGMRES cycles (Alg. 2); 1: RHOSVD-Tucker GMRES, full
    # Arnoldi (Alg. 1), which takes no sketch S (pass None)
    method: int = 0

    def struct(self, s: int, x0: Optional[Tucker] = None):
        p = TkSgmresParams()
        p.form, p.tol, p.eta, p.maxiter, p.max_restarts = self.form, self.tol, self.eta, self.maxiter, self.max_restarts
        p.k_trunc, p.rank_cap, p.oversample, p.s = self.k_trunc, self.rank_cap, self.oversample, s
        p.eps_trunc, p.eps_min, p.tol_inner_floor = self.eps_trunc, self.eps_min, self.tol_inner_floor
        p.tikhonov = int(self.tikhonov)
        p.method = int(self.method)
        keep = []
        if x0 is not None:
            xs = x0.struct()
            keep.append(xs)
            p.x0 = C.pointer(xs)
        p.precond_q = int(self.precond_q)
        if self.precond_q > 0:
            if self.precond is None:
                raise ValueError("precond_q > 0 needs the eigenpairs in `precond`")
            Vs, lams = self.precond
            va, la = _ptr_array(Vs), _ptr_array(lams)
            keep += [va, la]
            p.precond_V = va
            p.precond_lambda = la
        return p, keep


def precond_tensors(V: Sequence[np.ndarray], lam: Sequence[np.ndarray], device="cuda"):
    """Uploads per-mode eigenpairs (V_k n_k x n_k, lambda_k) of the 1D operator
    for ``SolveParams.precond`` (column-major device layout)."""
    return ([torch.from_numpy(np.ascontiguousarray(np.asarray(v, dtype=np.float64).T)).to(device) for v in V],
            [torch.from_numpy(np.ascontiguousarray(np.asarray(l, dtype=np.float64))).to(device) for l in lam])


def _info(hist_cap: int):
    info = TkSgmresInfo()
    hs = (C.c_double * hist_cap)()
    ht = (C.c_double * hist_cap)()
    hr = (C.c_int32 * (hist_cap * TK_MAX_D))()
    hc = (C.c_double * hist_cap)()
    hl = (C.c_double * hist_cap)()
    info.hist_cap = hist_cap
    info.hist_sketched = hs
    info.hist_true = ht
    info.hist_ranks = hr
    info.hist_cycle_seconds = hc
    info.hist_lambda = hl
    return info, (hs, ht, hr, hc, hl)


def _info_dict(info, keep, d):
    hs, ht, hr, hc, hl = keep
    n = info.hist_len
    return dict(status=int(info.status), status_name=_abi.STATUS.get(int(info.status), "?"),
                iters=int(info.iters_total), cycles=int(info.cycles), true_relres=float(info.true_relres),
                seconds=float(info.seconds), hist=[hs[i] for i in range(n)],
                true_hist=[ht[i] for i in range(int(info.cycles))],
                cycle_seconds=[hc[i] for i in range(int(info.cycles))],
                ranks=[tuple(hr[i * TK_MAX_D + k] for k in range(d)) for i in range(n)],
                lam=[hl[i] for i in range(n)])


def _hist_cap(prm: SolveParams) -> int:
    return prm.maxiter * max(prm.max_restarts, 1) + 8


def solve(op: KronOp, b: Tucker, S, omega, prm: SolveParams, x0: Optional[Tucker] = None, workspace=None):
    """Restarted Tucker sGMRES (or full-Arnoldi GMRES with ``prm.method`` 1,
    where ``S`` may be None); returns ``(x, info)``."""
    lib = _abi.load()
    ops, k1 = op.struct(b.n)
    bst = b.struct()
    s = int(S[0].shape[0]) if S is not None else 0
    ps, k2 = prm.struct(s, x0)
    nb = C.c_size_t()
    check(lib.tsgmres_solve_workspace(C.byref(ops), C.byref(bst), C.byref(ps), C.byref(nb)))
    # a caller's workspace is used as given: one that is too small makes the
    # library fail with TK_ERR_WORKSPACE before anything is launched
    ws = workspace if workspace is not None else _workspace(nb.value, b.core.device)
    x = Tucker.empty(b.n, (prm.rank_cap,) * b.d, b.core.device)
    xs = x.struct()
    info, keep = _info(_hist_cap(prm))
    check(lib.tsgmres_solve(C.byref(ops), C.byref(bst), C.byref(ps), _ptr_array(S) if S is not None else None,
                            _ptr_array(omega), C.byref(xs),
                            C.byref(info), C.c_void_p(ws.data_ptr()), int(ws.numel() * ws.element_size()),
                            _stream()))
    x.ranks = tuple(int(xs.r[k]) for k in range(b.d))
    return x, _info_dict(info, keep, b.d)


def solve_workspace_bytes(op: KronOp, b: Tucker, s: int, prm: SolveParams) -> int:
    lib = _abi.load()
    ops, k1 = op.struct(b.n)
    bst = b.struct()
    ps, k2 = prm.struct(s)
    nb = C.c_size_t()
    check(lib.tsgmres_solve_workspace(C.byref(ops), C.byref(bst), C.byref(ps), C.byref(nb)))
    return int(nb.value)


def backward(op: KronOp, x: Tucker, xbar_blocks, S, omega, prm: SolveParams, want_dA: bool = True):
    """Adjoint solve and gradients; returns ``(lambda, dalpha, dA, info)`` with
    ``dA[j][k]`` row-major ``(n_k, n_k)`` tensors (None for identity factors)."""
    lib = _abi.load()
    ops, k1 = op.struct(x.n)
    xst = x.struct()
    bs, k3 = _blocks_struct(xbar_blocks)
    s = int(S[0].shape[0])
    ps, k2 = prm.struct(s)
    nb = C.c_size_t()
    check(lib.tsgmres_backward_workspace(C.byref(ops), C.byref(xst), C.byref(bs), C.byref(ps), C.byref(nb)))
    ws = _workspace(nb.value, x.core.device)
    lam = Tucker.empty(x.n, (prm.rank_cap,) * x.d, x.core.device)
    ls_ = lam.struct()
    dal = (C.c_double * op.nterms)()
    dA = [[None if A is None else torch.zeros_like(A) for A in As] for As in op.A] if want_dA else None
    dAp = _ptr_array([t for row in dA for t in row]) if want_dA else None
    info, keep = _info(_hist_cap(prm))
    check(lib.tsgmres_backward(C.byref(ops), C.byref(xst), C.byref(bs), C.byref(ps), _ptr_array(S),
                               _ptr_array(omega), C.byref(ls_), dal, dAp, C.byref(info), C.c_void_p(ws.data_ptr()),
                               nb.value, _stream()))
    lam.ranks = tuple(int(ls_.r[k]) for k in range(x.d))
    return lam, np.array([dal[j] for j in range(op.nterms)]), dA, _info_dict(info, keep, x.d)


def project_core(x: Tucker, U: Sequence[torch.Tensor]) -> torch.Tensor:
    """``x x_1 U_1^T ... x_d U_d^T`` (a ``(m,) * d`` tensor) for factors
    ``U_k`` of shape ``(m, n_k)`` (column-major n_k x m): the projected core
    of the multilinear Nystrom sketch with Psi_k = U_k, computed by
    ``tucker_mln_sketch``."""
    m = int(U[0].shape[0])
    if any(int(u.shape[0]) != m for u in U):
        raise ValueError("project_core needs factors of one width in every mode")
    core, _, _ = mln_sketch([(1.0, x)], U, 1 if m > 1 else m)
    return core


_OK_STATUS = (0, 2)   # converged, or exact in the Krylov space (lucky breakdown)


class TuckerSGMRESLoss(torch.autograd.Function):
    """``loss(alpha, G_b) = ||x - x_target||^2 / 2`` where ``L(alpha) x = b``
    is solved by Tucker sGMRES and ``b = G_b x_1 U_1 ... x_d U_d`` has the
    differentiable core ``b_core`` and the fixed factors of ``problem['b']``.
    The backward pass is the hand-written adjoint: one transposed solve
    ``L^T lambda = x - x_target`` and the contractions
    ``dl/dalpha_j = -<lambda, x x_k A_j^(k)>`` (``tsgmres_backward``) and
    ``dl/dG_b = lambda x_k U_k^T`` (dl/db = lambda, projected on b's factors).

    ``problem``: op (KronOp, its alphas are replaced by ``alpha``), b (Tucker,
    factors of one rank capacity), x_target (Tucker), S, omega, prm
    (SolveParams).  A solve that ends other than converged or in a lucky
    breakdown raises.  After ``backward`` the adjoint solution (dl/db as a
    Tucker tensor) is in ``problem['lambda']``."""

    @staticmethod
    def forward(ctx, alpha: torch.Tensor, b_core: torch.Tensor, problem: dict):
        op = KronOp([float(a) for a in alpha.detach().cpu().tolist()], problem["op"].A)
        b0 = problem["b"]
        if tuple(b_core.shape) != b0.rcap:
            raise ValueError("b_core must have the shape of problem['b'].core")
        b = Tucker(b_core.detach().to(dtype=torch.float64, device=b0.core.device).contiguous(), b0.U, b0.ranks)
        x, info = solve(op, b, problem["S"], problem["omega"], problem["prm"])
        if info["status"] not in _OK_STATUS:
            raise RuntimeError(f"forward solve ended with status {info['status_name']} "
                               f"(true relative residual {info['true_relres']:.3e})")
        xt = problem["x_target"]
        loss = 0.5 * norm([(1.0, x), (-1.0, xt)]) ** 2
        ctx.problem = problem
        ctx.op = op
        ctx.x = x
        ctx.b = b
        ctx.meta = (alpha.dtype, alpha.device, b_core.dtype, b_core.device)
        problem["x"] = x
        problem["forward_info"] = info
        return torch.tensor(loss, dtype=torch.float64, device=alpha.device)

    @staticmethod
    def backward(ctx, g):
        p = ctx.problem
        adt, adev, bdt, bdev = ctx.meta
        lam, dalpha, _, info = backward(ctx.op, ctx.x, [(1.0, ctx.x), (-1.0, p["x_target"])], p["S"], p["omega"],
                                        p["prm"], want_dA=False)
        if info["status"] not in _OK_STATUS:
            raise RuntimeError(f"adjoint solve ended with status {info['status_name']} "
                               f"(true relative residual {info['true_relres']:.3e})")
        p["lambda"] = lam
        p["backward_info"] = info
        gs = g.detach().to(torch.float64)
        dal = (torch.as_tensor(dalpha, dtype=torch.float64, device=gs.device) * gs).to(dtype=adt, device=adev)
        db = None
        if ctx.needs_input_grad[1]:
            db = (project_core(lam, ctx.b.U) * gs.to(lam.core.device)).to(dtype=bdt, device=bdev)
        return dal, db, None


KERNEL_CLASSES = {"gemm": 0, "jacobi": 1, "qr": 2, "krp": 3, "ls": 4, "eigvals": 5, "tikhonov": 6}


def kernel_timer(kind: str, enable: bool) -> None:
    """Enable/disable (and clear) HIP-event timing of one kernel class."""
    check(_abi.load().tk_kernel_timer(KERNEL_CLASSES[kind], int(enable)))


def kernel_timer_read(kind: str):
    """(launches, total kernel milliseconds, algorithmic flops, algorithmic
    bytes) since enabling."""
    n = C.c_int64()
    ms = C.c_double()
    fl = C.c_double()
    by = C.c_double()
    check(_abi.load().tk_kernel_timer_read(KERNEL_CLASSES[kind], C.byref(n), C.byref(ms), C.byref(fl),
                                           C.byref(by)))
    return int(n.value), float(ms.value), float(fl.value), float(by.value)


def launch_count() -> int:
    """Kernel launches the library has issued since it was loaded."""
    n = C.c_int64()
    check(_abi.load().tk_launch_count(C.byref(n)))
    return int(n.value)


def launch_latency(n: int = 2000) -> float:
    """Microseconds per launch of an empty kernel, n back to back on the
    current stream."""
    us = C.c_double()
    check(_abi.load().tk_launch_latency(int(n), _stream(), C.byref(us)))
    return float(us.value)


def rank_cert_count() -> tuple:
    """(tried, passed): per-mode rank certificates of the effective-rank rule
    on the current device since the library was loaded (waits for the
    device)."""
    tried, passed = C.c_int64(), C.c_int64()
    check(_abi.load().tk_rank_cert_count(C.byref(tried), C.byref(passed)))
    return int(tried.value), int(passed.value)


def storage_floats(n: Sequence[int], ranks: Sequence[int]) -> int:
    """Floats stored by a Tucker tensor: sum_k n_k r_k + prod_k r_k."""
    return int(sum(a * b for a, b in zip(n, ranks)) + np.prod(ranks))


# ---------------------------------------------------------------- multilinear Nystrom
@dataclasses.dataclass
class MlnParams:
    r: int = 32
    p: int = 32
    tol: float = 1e-8
    eta: float = 0.4
    maxiter: int = 60
    k_trunc: int = 2
    breakdown_tol: float = -1.0
    save_memory: bool = False
    r_sol: int = 0
    p_sol: int = 0
    tikhonov: bool = False   # projected Tikhonov with GCV (Sec. 4.3)
    # exponential-sum preconditioner (Sec. 3.4), as in ``SolveParams``: the
    # method is then flexible and keeps the sketches of Z_i = recover(sketch(M(V_i)))
    precond_q: int = 0
    precond: Optional[Tuple[list, list]] = None

    def struct(self):
        """The C struct and the objects it points into (keep them alive for the call)."""
        p = TkMlnParams()
        p.r, p.p, p.tol, p.eta, p.maxiter, p.k_trunc = self.r, self.p, self.tol, self.eta, self.maxiter, self.k_trunc
        p.breakdown_tol, p.save_memory, p.r_sol, p.p_sol = self.breakdown_tol, int(self.save_memory), self.r_sol, \
            self.p_sol
        p.tikhonov = int(self.tikhonov)
        keep = []
        p.precond_q = int(self.precond_q)
        if self.precond_q > 0:
            if self.precond is None:
                raise ValueError("precond_q > 0 needs the eigenpairs in `precond`")
            Vs, lams = self.precond
            va, la = _ptr_array(Vs), _ptr_array(lams)
            keep += [va, la]
            p.precond_V = va
            p.precond_lambda = la
        return p, keep


def mln_sketch(blocks, Psi: Sequence[torch.Tensor], r: int):
    """Multilinear Nystrom sketch of a block sum; returns ``(core, F, diag)``
    with core ``(r + p,) * d``, ``F[k]`` of shape ``(r, n_k)`` and the
    superdiagonal ``diag`` of the core (length ``r + p``)."""
    lib = _abi.load()
    bs, keep = _blocks_struct(blocks)
    x0 = blocks[0][1]
    dev = x0.core.device
    rt = int(Psi[0].shape[0])
    p = rt - int(r)
    core = torch.zeros((rt,) * x0.d, dtype=torch.float64, device=dev)
    F = [torch.zeros((r, nk), dtype=torch.float64, device=dev) for nk in x0.n]
    diag = torch.zeros(rt, dtype=torch.float64, device=dev)
    nb = C.c_size_t()
    check(lib.tucker_mln_sketch_workspace(C.byref(bs), int(r), p, C.byref(nb)))
    ws = _workspace(nb.value, dev)
    check(lib.tucker_mln_sketch(C.byref(bs), _ptr_array(Psi), int(r), p, C.c_void_p(core.data_ptr()), _ptr_array(F),
                                C.c_void_p(diag.data_ptr()), C.c_void_p(ws.data_ptr()), nb.value, _stream()))
    return core, F, diag


def mln_recover(core: torch.Tensor, F: Sequence[torch.Tensor], Psi: Sequence[torch.Tensor], r: int) -> Tucker:
    """Multilinear Nystrom recovery of a sketched tensor (rank capacity r)."""
    lib = _abi.load()
    d = core.dim()
    rt = int(Psi[0].shape[0])
    n = tuple(int(P.shape[1]) for P in Psi)
    out = Tucker.empty(n, (r,) * d, core.device)
    os_ = out.struct()
    nn = (C.c_int64 * TK_MAX_D)(*(list(n) + [1] * (TK_MAX_D - d)))
    nb = C.c_size_t()
    check(lib.tucker_mln_recover_workspace(d, nn, int(r), rt - int(r), C.byref(nb)))
    ws = _workspace(nb.value, core.device)
    check(lib.tucker_mln_recover(C.c_void_p(core.data_ptr()), _ptr_array(F), _ptr_array(Psi), int(r), rt - int(r),
                                 C.byref(os_), C.c_void_p(ws.data_ptr()), nb.value, _stream()))
    out.ranks = tuple(int(os_.r[k]) for k in range(d))
    return out


def mln_solve_workspace_bytes(op: KronOp, b: Tucker, prm: MlnParams) -> int:
    lib = _abi.load()
    ops, k1 = op.struct(b.n)
    bst = b.struct()
    ps, kp = prm.struct()
    nb = C.c_size_t()
    check(lib.tsgmres_mln_solve_workspace(C.byref(ops), C.byref(bst), C.byref(ps), C.byref(nb)))
    return int(nb.value)


def mln_solve(op: KronOp, b: Tucker, Psi: Sequence[torch.Tensor], prm: MlnParams, workspace=None):
    """MLN-Tucker sGMRES; returns ``(x, info)``."""
    lib = _abi.load()
    ops, k1 = op.struct(b.n)
    bst = b.struct()
    ps, kp = prm.struct()
    nb = C.c_size_t()
    check(lib.tsgmres_mln_solve_workspace(C.byref(ops), C.byref(bst), C.byref(ps), C.byref(nb)))
    # a caller's workspace is used as given: one that is too small makes the
    # library fail with TK_ERR_WORKSPACE before anything is launched
    ws = workspace if workspace is not None else _workspace(nb.value, b.core.device)
    x = Tucker.empty(b.n, (prm.r,) * b.d, b.core.device)
    xs = x.struct()
    info, keep = _info(prm.maxiter + 8)
    check(lib.tsgmres_mln_solve(C.byref(ops), C.byref(bst), C.byref(ps), _ptr_array(Psi), C.byref(xs), C.byref(info),
                                C.c_void_p(ws.data_ptr()), nb.value, _stream()))
    x.ranks = tuple(int(xs.r[k]) for k in range(b.d))
    return x, _info_dict(info, keep, b.d)


# ---------------------------------------------------------------- projected Tikhonov
def projected_tikhonov(M: torch.Tensor, b: torch.Tensor, lam: Optional[float] = None):
    """Regularised least squares argmin ||M y - b||^2 + lambda^2 ||y||^2 on
    the device (Sec. 4.3): ``M`` is an (s, k) FP64 CUDA tensor, ``b`` length
    s; ``lam`` None chooses lambda by GCV.  Returns (y, lambda, ||M y - b|| /
    ||b||)."""
    lib = _abi.load()
    if M.dim() != 2 or M.dtype != torch.float64 or not M.is_cuda:
        raise ValueError("M must be a 2D float64 CUDA tensor")
    s, k = int(M.shape[0]), int(M.shape[1])
    if b.shape != (s,) or b.dtype != torch.float64 or b.device != M.device:
        raise ValueError("b must be a float64 vector of length s on M's device")
    Mc = M.t().contiguous()            # column-major s x k
    bc = b.contiguous()
    nb = C.c_size_t()
    check(lib.tsgmres_projected_tikhonov_workspace(s, k, C.byref(nb)))
    ws = _workspace(nb.value, M.device)
    y = torch.empty(k, dtype=torch.float64, device=M.device)
    out = torch.empty(2, dtype=torch.float64, device=M.device)
    check(lib.tsgmres_projected_tikhonov(C.c_void_p(Mc.data_ptr()), C.c_void_p(bc.data_ptr()), s, k,
                                         -1.0 if lam is None else float(lam), C.c_void_p(y.data_ptr()),
                                         C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()), nb.value,
                                         _stream()))
    o = out.cpu()
    return y, float(o[0]), float(o[1])
