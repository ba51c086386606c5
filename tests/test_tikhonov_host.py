"""Host logic of projected Tikhonov (no GPU: workspace queries and argument
checks, which plan without launching anything)."""
import ctypes as C
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2608_11091_amd", "libtsgmres.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")

torch = pytest.importorskip("torch")


def _lib():
    from paper_2608_11091_amd import _abi
    return _abi.load()


@pytest.mark.parametrize("s,k,ok", [(10, 1, True), (256, 64, True), (64, 65, False), (257, 8, False),
                                    (8, 9, False), (8, 0, False)])
def test_workspace_query_limits(s, k, ok):
    nb = C.c_size_t()
    rc = _lib().tsgmres_projected_tikhonov_workspace(s, k, C.byref(nb))
    assert (rc == 0) == ok
    if ok:
        # Householder vectors, R, Q^T b, y, residuals, lambdas and small scalars
        assert nb.value >= 8 * (s * k + k * k + s + 3 * k)


def _op_b(n=12):
    import paper_2608_11091_amd as tk
    from workloads import laplacian_1d
    L = laplacian_1d(n)
    op = tk.KronOp.from_terms([(1.0, [L if j == k else None for j in range(3)]) for k in range(3)], device="cpu")
    b = tk.Tucker.from_numpy(np.ones((1, 1, 1)), [np.ones((n, 1))] * 3, device="cpu")
    return tk, op, b


def test_solve_rejects_bad_tikhonov_flag():
    tk, op, b = _op_b()
    from paper_2608_11091_amd._abi import TkError
    with pytest.raises(TkError):
        tk.solve_workspace_bytes(op, b, 40, tk.SolveParams(tikhonov=2, rank_cap=8, maxiter=10))
    with pytest.raises(TkError):
        tk.mln_solve_workspace_bytes(op, b, tk.MlnParams(r=8, p=8, tikhonov=3))


def test_backward_rejects_regularised_solve():
    # the adjoint gradients are those of an unregularised solve
    tk, op, b = _op_b()
    from paper_2608_11091_amd import _abi
    lib = _lib()
    ops, k1 = op.struct(b.n)
    bst = b.struct()
    ps, k2 = tk.SolveParams(tikhonov=True, rank_cap=8, maxiter=10).struct(40)
    xb = _abi.TkBlockSum()
    xb.nblocks = 1
    xb.coef = (C.c_double * 1)(1.0)
    xb.blocks = C.pointer(bst)
    nb = C.c_size_t()
    rc = lib.tsgmres_backward_workspace(C.byref(ops), C.byref(bst), C.byref(xb), C.byref(ps), C.byref(nb))
    assert rc == -7 and b"unregularised" in lib.tk_last_error()
