"""Host argument checks of the full-Arnoldi method (no GPU: the checks run
before any planning)."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2608_11091_amd", "libtsgmres.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")

torch = pytest.importorskip("torch")


def _op_b(n=12):
    import paper_2608_11091_amd as tk
    from workloads import laplacian_1d
    L = laplacian_1d(n)
    op = tk.KronOp.from_terms([(1.0, [L if j == k else None for j in range(3)]) for k in range(3)], device="cpu")
    b = tk.Tucker.from_numpy(np.ones((1, 1, 1)), [np.ones((n, 1))] * 3, device="cpu")
    return tk, op, b


@pytest.mark.parametrize("kw,code", [
    (dict(method=2), -1),                                   # unknown method
    (dict(method=1, precond_q=4, precond=([], [])), -7),    # no preconditioned full Arnoldi
])
def test_solve_rejects(kw, code):
    tk, op, b = _op_b()
    from paper_2608_11091_amd._abi import TkError
    with pytest.raises(TkError) as e:
        tk.solve_workspace_bytes(op, b, 40, tk.SolveParams(rank_cap=8, maxiter=10, **kw))
    assert e.value.code == code


def test_backward_rejects_full_arnoldi():
    import ctypes as C
    tk, op, b = _op_b()
    from paper_2608_11091_amd import _abi
    lib = _abi.load()
    ops, k1 = op.struct(b.n)
    bst = b.struct()
    ps, k2 = tk.SolveParams(method=1, rank_cap=8, maxiter=10).struct(40)
    xb = _abi.TkBlockSum()
    xb.nblocks = 1
    xb.coef = (C.c_double * 1)(1.0)
    xb.blocks = C.pointer(bst)
    nb = C.c_size_t()
    rc = lib.tsgmres_backward_workspace(C.byref(ops), C.byref(bst), C.byref(xb), C.byref(ps), C.byref(nb))
    assert rc == -7 and b"method 0" in lib.tk_last_error()
