"""Host logic of the multilinear Nystrom entry points (no GPU: only the
workspace queries, which plan without launching anything, and their argument
checks)."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2608_11091_amd", "libtsgmres.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")

torch = pytest.importorskip("torch")


def _problem(n=64, d=3):
    import paper_2608_11091_amd as tk
    from workloads import laplacian_1d
    L = laplacian_1d(n)
    terms = [(1.0, [L if j == k else None for j in range(d)]) for k in range(d)]
    op = tk.KronOp.from_terms(terms, device="cpu")
    b = tk.Tucker.from_numpy(np.ones((1,) * d), [np.ones((n, 1))] * d, device="cpu")
    return tk, op, b


def _sketch_bytes(n, d, r, rt):
    # one stored sketch: the (r + p)^d core and d factor sketches, 256-byte aligned
    al = lambda b: (b + 255) // 256 * 256
    return al(8 * rt ** d) + d * al(8 * n * r)


def test_mln_solve_workspace_memory_efficient_variant():
    # save_memory keeps kt + 2 full sketches plus truncated copies, instead of
    # maxiter + 1 full sketches (Sec. 3.3, memory-efficient variant)
    tk, op, b = _problem()
    n, d, r, p, mx, kt, rs, ps = 64, 3, 16, 16, 30, 2, 4, 4
    full = tk.mln_solve_workspace_bytes(op, b, tk.MlnParams(r=r, p=p, maxiter=mx, k_trunc=kt))
    save = tk.mln_solve_workspace_bytes(op, b, tk.MlnParams(r=r, p=p, maxiter=mx, k_trunc=kt, save_memory=True,
                                                            r_sol=rs, p_sol=ps))
    big = _sketch_bytes(n, d, r, r + p)
    small = _sketch_bytes(n, d, rs, rs + ps)
    expect = (mx + 1 - (kt + 2)) * big - (mx + 1) * small
    # plus the smaller final-sum sketch and the smaller temporaries of the
    # final recovery (at most a few more full sketches' worth)
    assert expect <= full - save <= expect + 3 * big
    # the full-memory workspace holds every stored sketch
    assert full >= (mx + 1) * big


@pytest.mark.parametrize("kw,code", [
    (dict(r=65, p=0), -7),                         # target rank above 64
    (dict(r=32, p=300), -7),                       # r + p above 256
    (dict(r=8, p=8, maxiter=65), -7),              # maxiter above 64
    (dict(r=8, p=8, k_trunc=0), -1),
    (dict(r=8, p=8, save_memory=True, r_sol=9, p_sol=0), -1),   # r_sol above r
    (dict(r=8, p=8, save_memory=True, r_sol=4, p_sol=13), -1),  # r_sol + p_sol above r + p
])
def test_mln_solve_rejects_out_of_range(kw, code):
    tk, op, b = _problem(16)
    from paper_2608_11091_amd._abi import TkError
    with pytest.raises(TkError) as e:
        tk.mln_solve_workspace_bytes(op, b, tk.MlnParams(**kw))
    assert e.value.code == code


def test_mln_solve_rejects_rhs_rank_above_r():
    import paper_2608_11091_amd as tk
    from paper_2608_11091_amd._abi import TkError
    _, op, _ = _problem(16)
    rng = np.random.default_rng(0)
    b = tk.Tucker.from_numpy(rng.standard_normal((5, 5, 5)), [rng.standard_normal((16, 5))] * 3, device="cpu")
    with pytest.raises(TkError) as e:
        tk.mln_solve_workspace_bytes(op, b, tk.MlnParams(r=4, p=4))
    assert e.value.code == -3


def test_mln_sketch_and_recover_workspace_queries():
    # host-only planning of the sketch and recovery calls (every output
    # pointer is only recorded); sizes grow with the sketch width
    import ctypes as C
    import paper_2608_11091_amd as tk
    from paper_2608_11091_amd import _abi, api
    rng = np.random.default_rng(0)
    n = (77, 70, 65)
    X = tk.Tucker.from_numpy(rng.standard_normal((5, 7, 6)), [rng.standard_normal((nk, rk))
                                                               for nk, rk in zip(n, (5, 7, 6))], device="cpu",
                             rcap=(8, 8, 8))
    lib = _abi.load()
    bs, keep = api._blocks_struct([(1.0, X), (-0.5, X)])
    sizes = []
    for r, p in ((20, 12), (20, 44)):
        nb = C.c_size_t()
        assert lib.tucker_mln_sketch_workspace(C.byref(bs), r, p, C.byref(nb)) == 0
        sizes.append(nb.value)
    assert sizes[1] > sizes[0] > 0
    nn = (C.c_int64 * 4)(*n, 1)
    nb = C.c_size_t()
    assert lib.tucker_mln_recover_workspace(3, nn, 20, 12, C.byref(nb)) == 0
    # at least the (r + p)^(d-1) r ping-pong buffers of the core contraction
    assert nb.value >= 2 * 8 * 32 * 32 * 20
    assert lib.tucker_mln_recover_workspace(3, nn, 65, 0, C.byref(nb)) == -7


def test_flexible_mln_workspace_and_checks():
    # The flexible method (Sec. 3.4) keeps one sketch of every Z_i besides the
    # basis sketches: maxiter more full sketches, or maxiter truncated ones
    # plus one full sketch with save_memory.  q outside [0, 400] and a
    # missing eigenpair list are rejected before anything is planned.
    tk, op, b = _problem()
    from paper_2608_11091_amd._abi import TkError
    from workloads import laplacian_eigenpairs
    n, d, r, p, mx, kt, rs, ps = 64, 3, 16, 16, 30, 2, 4, 4
    pc = tk.precond_tensors(*laplacian_eigenpairs((n,) * d), device="cpu")
    big, small = _sketch_bytes(n, d, r, r + p), _sketch_bytes(n, d, rs, rs + ps)
    plain = tk.mln_solve_workspace_bytes(op, b, tk.MlnParams(r=r, p=p, maxiter=mx, k_trunc=kt))
    flex = tk.mln_solve_workspace_bytes(op, b, tk.MlnParams(r=r, p=p, maxiter=mx, k_trunc=kt, precond_q=16,
                                                            precond=pc))
    assert flex - plain >= mx * big
    kw = dict(r=r, p=p, maxiter=mx, k_trunc=kt, save_memory=True, r_sol=rs, p_sol=ps)
    plain_s = tk.mln_solve_workspace_bytes(op, b, tk.MlnParams(**kw))
    flex_s = tk.mln_solve_workspace_bytes(op, b, tk.MlnParams(**kw, precond_q=16, precond=pc))
    # save_memory stores maxiter truncated Z sketches and one full one (and
    # drops the truncated copies of the basis sketches, which the flexible
    # solution does not use): about maxiter - 1 full sketches fewer, less a
    # difference in the arena's peak of temporaries below one full sketch
    assert (flex - plain) - (flex_s - plain_s) >= (mx - 3) * big
    with pytest.raises(ValueError):
        tk.MlnParams(r=4, p=4, precond_q=8).struct()
    for q in (-1, 401):
        with pytest.raises(TkError) as e:
            tk.mln_solve_workspace_bytes(op, b, tk.MlnParams(r=4, p=4, precond_q=q, precond=pc))
        assert e.value.code == -1
