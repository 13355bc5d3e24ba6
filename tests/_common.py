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
