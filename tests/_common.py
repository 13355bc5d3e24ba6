"""Helpers shared by the test modules (no method arithmetic)."""
import numpy as np


def oracle_problem(pr):
    import oracle
    return oracle.problem_from_dict(pr)


def rel_l2(got, ref):
    """max over right-hand sides of ||got - ref||_2 / ||ref||_2 (leading axis = RHS)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.ndim == 1 or ref.ndim == 1:
        got, ref = got.reshape(1, -1), ref.reshape(1, -1)
    g = got.reshape(got.shape[0], -1)
    r = ref.reshape(ref.shape[0], -1)
    return float(np.max(np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)))


def fp64_bar(Gp, Gq, x, transpose=False, c=10.0, floor=1e-12):
    """The FP64 bar for products whose entries come from the FP64 closed
    forms: the larger of ``floor`` and ``c`` times the relative error that the
    oracle's own plain-FP64 entries (Gp, evaluated from the geometry in
    double) make against the exact ones (Gq, __float128 rounded once) on the
    same product.  For distant prisms the corner sums cancel, so every FP64
    evaluation of the closed forms carries this error; the bar admits no more
    than ``c`` times it."""
    x = np.asarray(x, dtype=np.float64).ravel()
    if transpose:
        a, b = Gp.T @ x, Gq.T @ x
    else:
        a, b = Gp @ x, Gq @ x
    return max(floor, c * float(np.linalg.norm(a - b) / np.linalg.norm(b)))
