"""Measured parity bounds for trajectories that amplify rounding.

Where the rank cap binds, the kept subspace is not determined beyond
rounding (the cut falls inside a continuum of singular values), and the
truncated short recurrence amplifies any rounding-level difference over the
following iterations and cycles.  The bound for the GPU against the oracle is
then measured, not asserted, from the oracle's own spread over rounding-level
choices that are all valid:
  * the right-hand side's core changed by one unit roundoff (2^-52, iid signs);
  * the range-finder basis of the cycle's RoundSums taken from shifted
    Cholesky-QR3 instead of Householder QR (Sec. 3.1 fixes range(Y_k), not
    its basis; the GPU's FP64 form uses Cholesky-QR3 there);
  * for the FP32 form, every RoundSum operand, operator factor, sketch and
    the right-hand side rounded to FP32 (the FP32 form rounds its operands on
    entry);
  * the GPU's own spread: the same GPU solve on the right-hand side changed
    by one unit roundoff of the form (2^-52, or 2^-24 for the FP32 form),
    which measures how strongly the form's own arithmetic is amplified.
The GPU may deviate from the oracle by at most ten times the largest of these
spreads (running maximum along the trajectory), and always by the FP64
parity bound 1e-10 (1e-4 for the FP32 form, its RoundSum bound).  The FP32
form's own arithmetic seeds the amplification far above its operand
rounding, so its trajectories are held to these bounds only before the
amplification starts and at the end of the cycle (true residual, solution)."""
import numpy as np

import oracle as O


def perturbed_rhs(B: O.Tucker, seed: int = 99, rel: float = 2.0 ** -52) -> O.Tucker:
    rng = np.random.default_rng(seed)
    return O.Tucker(B.core * (1.0 + rel * rng.choice([-1.0, 1.0], size=B.core.shape)), B.U)


def rel_spread(h_ref, h_pert):
    """Relative difference of two histories over their common length."""
    h_ref, h_pert = np.asarray(h_ref), np.asarray(h_pert)
    m = min(len(h_ref), len(h_pert))
    return np.abs(h_pert[:m] - h_ref[:m]) / np.abs(h_ref[:m])


def bound_from_spreads(spreads, m, floor=1e-10):
    """10x the running maximum (with one iteration of lookahead) of the
    largest of the given spread arrays, over the first m iterations."""
    sp = np.zeros(m)
    for a in spreads:
        a = np.asarray(a)[:m]
        sp[:len(a)] = np.maximum(sp[:len(a)], a)
    run = np.maximum.accumulate(sp)
    ahead = np.concatenate([run[1:], run[-1:]])
    return np.maximum(floor, 10.0 * ahead)


def history_bound(h_ref, h_perts, floor=1e-10):
    """Per-iteration allowance: 10x the running maximum of the oracle's own
    relative spread (the largest over the perturbed runs `h_perts`, one array
    or a list of arrays) up to the next iteration -- the onset of the
    amplification can come one iteration earlier on another valid trajectory
    -- never below `floor`."""
    h_ref = np.asarray(h_ref)
    if len(h_perts) and np.ndim(h_perts[0]) == 0:
        h_perts = [h_perts]
    m = min([len(h_ref)] + [len(h) for h in h_perts])
    spread = np.zeros(m)
    for h in h_perts:
        h = np.asarray(h)
        spread = np.maximum(spread, np.abs(h[:m] - h_ref[:m]) / np.abs(h_ref[:m]))
    run = np.maximum.accumulate(spread)
    ahead = np.concatenate([run[1:], run[-1:]])
    return np.maximum(floor, 10.0 * ahead)


def f32(a):
    """Round to FP32 and back (None passes through)."""
    return None if a is None else np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def fp32_operands(terms, B, S, Omega):
    """The problem with every operand rounded to FP32."""
    return ([(a, [f32(A) for A in As]) for a, As in terms], O.Tucker(f32(B.core), [f32(u) for u in B.U]),
            [f32(x) for x in S], [f32(x) for x in Omega])


def first_divergence(h_gpu, h_ref, floor=1e-10):
    """Index of the first iteration whose relative difference exceeds `floor`
    (None when none does)."""
    h_gpu, h_ref = np.asarray(h_gpu), np.asarray(h_ref)
    m = min(len(h_gpu), len(h_ref))
    d = np.abs(h_gpu[:m] - h_ref[:m]) / np.abs(h_ref[:m])
    idx = np.nonzero(d > floor)[0]
    return int(idx[0]) if idx.size else None


def cholesky_qr3(Y: np.ndarray) -> np.ndarray:
    """Another valid orthonormal basis of range(Y) (Sec. 3.1 fixes the range,
    not the basis): three Cholesky-QR passes, the first shifted by
    11 (n s + s(s+1)) u tr(Y^T Y); a pivot at or below 1e-30 tr (second pass)
    or 1/4 (third pass, nearly orthonormal input) marks a dependent column,
    which comes out as a zero column.  Used to measure how much the choice of
    basis alone moves a trajectory."""
    u = 2.0 ** -53
    n, s = Y.shape
    Q = Y.copy()
    for pas in range(3):
        G = Q.T @ Q
        tr = float(np.trace(G))
        if pas == 0:
            G = G + 11.0 * (n * s + s * (s + 1)) * u * tr * np.eye(s)
        thr = 0.0 if pas == 0 else (1e-30 * tr if pas == 1 else 0.25)
        R = np.zeros((s, s))
        live = np.zeros(s, dtype=bool)
        for j in range(s):
            piv = G[j, j] - R[:j, j] @ R[:j, j]
            if piv <= thr or not np.isfinite(piv):
                continue
            live[j] = True
            R[j, j] = np.sqrt(piv)
            R[j, j + 1:] = (G[j, j + 1:] - R[:j, j] @ R[:j, j + 1:]) / R[j, j]
        Qn = np.zeros_like(Q)
        # Q R = Y restricted to the live columns: forward substitution by columns
        for j in range(s):
            if not live[j]:
                continue
            v = Q[:, j] - Qn[:, :j] @ R[:j, j]
            Qn[:, j] = v / R[j, j]
        Q = Qn
    return Q
