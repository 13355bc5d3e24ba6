"""User-supplied kernels (BTTB_USER_TABLE): the caller's entries per layer
and cell offset, embedded, transformed and multiplied by the library,
against the oracle's dense matrix of the same entries."""
import numpy as np
import pytest

import workloads as W
from _common import oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

SHAPES = [
    W.problem(W.TABLE, 13, 11, 5, 0, 3, 4, 1, dx=1.0, dy=1.0, dz=1.0),
    W.problem(W.TABLE, 23, 17, 4, 3, 2, 5, 4, dx=1.0, dy=1.0, dz=1.0),
    W.problem(W.TABLE, 1, 6, 2, 0, 0, 2, 1, dx=1.0, dy=1.0, dz=1.0),
]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _table_shape(pr):
    nx, ny, nz = W.dims(pr)
    return nz, pr["sy"] + ny - 1, pr["sx"] + nx - 1


def _run(torch, pr, prec, table):
    from paper_1912_06976_amd import Plan
    plan = Plan(pr, prec).generate(table=torch.tensor(table, dtype=torch.float64, device="cuda"))
    m = W.normal_model(pr, 71)
    v = W.normal_data(pr, 72)
    d = plan.forward(torch.tensor(m, dtype=plan.dtype, device="cuda"))
    t = plan.transpose(torch.tensor(v, dtype=plan.dtype, device="cuda"))
    torch.cuda.synchronize()
    return plan, m, v, d.double().cpu().numpy(), t.double().cpu().numpy()


@pytest.mark.parametrize("k", range(len(SHAPES)))
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_random_table_matches_dense(torch_cuda, k, prec, tol):
    import oracle
    pr = SHAPES[k]
    print("table", k, prec, flush=True)
    table = np.random.default_rng(700 + k).standard_normal(_table_shape(pr))
    plan, m, v, d, t = _run(torch_cuda, pr, prec, table)
    assert plan.spectrum_form == "complex"
    G = oracle.dense_from_table(pr, table)
    assert rel_l2(d.ravel(), G @ m.ravel()) <= tol
    assert rel_l2(t.ravel(), G.T @ v.ravel()) <= tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_even_table_in_both_spectrum_forms(torch_cuda, prec, tol):
    # an even kernel h(|dx|, |dy|), declared so: real even spectra read the
    # mirror of offsets the table has on one side only (pxl != pxr)
    import oracle
    pr = dict(W.problem(W.TABLE, 23, 17, 4, 3, 2, 5, 4, dx=1.0, dy=1.0, dz=1.0))
    nz, wy, wx = _table_shape(pr)
    rng = np.random.default_rng(77)
    ax = np.abs(np.arange(wx) - (pr["sx"] - 1 + pr["pxl"]))
    ay = np.abs(np.arange(wy) - (pr["sy"] - 1 + pr["pyl"]))
    base = rng.standard_normal((nz, ay.max() + 1, ax.max() + 1))
    table = np.ascontiguousarray(base[:, ay[:, None], ax[None, :]])
    G = oracle.dense_from_table(pr, table)
    for form in ("real_even", "complex"):
        plan, m, v, d, t = _run(torch_cuda, dict(pr, spectrum_form=form), prec, table)
        assert plan.spectrum_form == form
        assert rel_l2(d.ravel(), G @ m.ravel()) <= tol
        assert rel_l2(t.ravel(), G.T @ v.ravel()) <= tol


def test_gravity_entries_as_table_equal_builtin_kernel(torch_cuda):
    # the exact gravity entries supplied as a table give the gravity products
    import oracle
    pr = W.small_gravity()
    P = oracle_problem(pr)
    tq, _ = oracle.offset_table_quad(P)
    G = oracle.dense_G_quad(P)
    prt = dict(pr, kind=W.TABLE)
    plan, m, v, d, t = _run(torch_cuda, prt, "fp64", tq)
    assert rel_l2(d.ravel(), G @ m.ravel()) <= 1e-13
    assert rel_l2(t.ravel(), G.T @ v.ravel()) <= 1e-13


def test_table_plan_errors(torch_cuda):
    import paper_1912_06976_amd as B
    torch = torch_cuda
    pr = SHAPES[0]
    plan = B.Plan(pr, "fp64")
    with pytest.raises(ValueError):
        plan.generate()
    spectra = torch.empty(plan.spectra_bytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.BttbError):
        B.bttb_kernel_generate(plan.handle, spectra, plan.workspace(1))
    g = B.Plan(W.small_gravity(), "fp64")
    table = torch.zeros(_table_shape(W.small_gravity()), dtype=torch.float64, device="cuda")
    with pytest.raises(B.BttbError):
        B.bttb_kernel_generate_table(g.handle, table, spectra, g.workspace(1))
