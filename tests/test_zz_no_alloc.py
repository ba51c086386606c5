"""The allocation-free Khatri-Rao sketch entry point (tucker_sketch_noalloc)
against the workspace entry point (tucker_sketch) and the oracle, through the
C ABI: two calls in a row on the shared static scratch, the second with a
smaller input, in both forms; and an input too large for the scratch is
rejected before anything is launched."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tk():
    import paper_2608_11091_amd as tk
    tk.load()
    return tk


def _cm(M):
    return torch.from_numpy(np.ascontiguousarray(M.T)).cuda()


def _case(seed, n, r, nb, s):
    rng = np.random.default_rng(seed)
    blocks = []
    for _ in range(nb):
        U = [rng.standard_normal((nk, rk)) for nk, rk in zip(n, r)]
        blocks.append((float(rng.uniform(-2, 2)), O.Tucker(rng.standard_normal(tuple(r)), U)))
    S = [rng.standard_normal((nk, s)) for nk in n]
    return blocks, S


def _check(tk, blocks, S, form, tol_oracle):
    gb = [(c, tk.Tucker.from_numpy(X.core, X.U)) for c, X in blocks]
    St = [_cm(x) for x in S]
    ref = tk.sketch(gb, St, form=form).cpu().numpy()
    out = torch.full((len(ref),), float("nan"), dtype=torch.float64, device="cuda")
    got = tk.sketch_noalloc(gb, St, out, form=form).cpu().numpy()
    want = O.sketch_krp(blocks, S)
    print("form", form, "n", blocks[0][1].n, "s", len(ref), "max |noalloc - workspace|", np.max(np.abs(got - ref)),
          flush=True)
    # same kernels on the same inputs: identical to the workspace entry point
    assert np.array_equal(got, ref)
    assert np.linalg.norm(got - want) <= tol_oracle * np.linalg.norm(want)


@pytest.mark.parametrize("form,tol", [(0, 1e-12), (1, 1e-5)])
def test_noalloc_sketch_two_calls(tk, form, tol):
    # first call: the deblurring workload's shape (n = 512, rank 48, s = 120,
    # three blocks as in the orthogonalisation sum); second call smaller and
    # ragged (n = 77, 70, 65), reusing the scratch the first call left behind
    b1, S1 = _case(1, (512, 512, 512), (48, 48, 48), 3, 120)
    _check(tk, b1, S1, form, tol)
    b2, S2 = _case(2, (77, 70, 65), (5, 7, 6), 2, 130)
    _check(tk, b2, S2, form, tol)


def test_noalloc_sketch_rejects_oversized_input(tk):
    # d = 4, rank 64: one core alone is 128 MiB, above the 64 MiB scratch
    n, r = (128, 128, 128, 128), (64, 64, 64, 64)
    core = torch.zeros(r, dtype=torch.float64, device="cuda")
    U = [torch.zeros((64, 128), dtype=torch.float64, device="cuda") for _ in n]
    X = tk.Tucker(core=core, U=U, ranks=r)
    S = [torch.zeros((16, 128), dtype=torch.float64, device="cuda") for _ in n]
    out = torch.full((16,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(tk.TkError) as e:
        tk.sketch_noalloc([(1.0, X)], S, out)
    assert e.value.code == -4 and "static maximum" in str(e.value)
    assert bool((out == 7.0).all())
