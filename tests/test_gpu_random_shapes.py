"""Seeded random small problems (both kernels, both spectrum forms, both
precisions, asymmetric paddings, raised stations, several right-hand sides)
against the oracle's dense matrix of exact entries."""
import numpy as np
import pytest

import workloads as W
from _common import fp64_bar, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

NCASES = 24
TOL = {"fp64": 1e-12, "fp32": 2e-5}


def _case(k):
    rng = np.random.default_rng(9000 + k)
    sx, sy = (int(v) for v in rng.integers(1, 41, size=2))
    pads = [int(v) for v in rng.integers(0, 6, size=4)]
    nz = int(rng.integers(1, 7))
    d = float(rng.choice([10.0, 25.0, 50.0]))
    kw = dict(dx=d, dy=float(rng.choice([d, 2 * d])), dz=d / 2, h=float(rng.choice([0.0, 3.0])))
    kind = W.GRAVITY if k % 2 == 0 else W.MAGNETIC
    if kind == W.MAGNETIC:
        kw.update(incl=float(rng.uniform(-90, 90)), decl=float(rng.uniform(-180, 180)), field_nT=47000.0)
    pr = W.problem(kind, sx, sy, nz, *pads, **kw)
    if kind == W.GRAVITY and k % 4 == 2:
        pr["spectrum_form"] = "complex"
    prec = "fp64" if k % 3 else "fp32"
    nrhs = 1 + k % 3
    return pr, prec, nrhs


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _products(torch, plan, m, v):
    d = plan.forward(torch.tensor(m, dtype=plan.dtype, device="cuda"))
    t = plan.transpose(torch.tensor(v, dtype=plan.dtype, device="cuda"))
    torch.cuda.synchronize()
    return d.double().cpu().numpy(), t.double().cpu().numpy()


@pytest.mark.parametrize("k", range(NCASES))
def test_random_shape(torch_cuda, k):
    import oracle
    from paper_1912_06976_amd import Plan
    torch = torch_cuda
    pr, prec, nrhs = _case(k)
    print("random case", k, pr["kind"], pr["sx"], pr["sy"], pr["nz"], prec, nrhs, flush=True)
    P = oracle_problem(pr)
    G = oracle.dense_G_quad(P)
    Gp = oracle.dense_G(P)
    m = W.normal_model(pr, 9100 + k, nrhs=nrhs).reshape(nrhs, -1)
    v = W.normal_data(pr, 9200 + k, nrhs=nrhs).reshape(nrhs, -1)
    shape_m = (nrhs,) + W.normal_model(pr, 0).shape
    shape_v = (nrhs, pr["sy"], pr["sx"])
    tol = TOL[prec]

    # 1. generated entries.  The closed-form corner sums are evaluated in
    # FP64; for distant prisms they cancel.  FP64 is held to the larger of the
    # bar and 10x the error the oracle's own plain-FP64 entries make on the
    # same product (fp64_bar).
    plan = Plan(pr, prec).generate()
    d, t = _products(torch, plan, m.reshape(shape_m), v.reshape(shape_v))
    d, t = d.reshape(nrhs, -1), t.reshape(nrhs, -1)
    for q in range(nrhs):
        bf = fp64_bar(Gp, G, m[q]) if prec == "fp64" else tol
        bt = fp64_bar(Gp, G, v[q], transpose=True) if prec == "fp64" else tol
        assert rel_l2(d[q], G @ m[q]) <= bf, q
        assert rel_l2(t[q], G.T @ v[q]) <= bt, q

    # 2. the same products from the exact entries, supplied as a table:
    # no entry rounding left, so the bar holds as stated
    tq, _ = oracle.offset_table_quad(P)
    form = plan.spectrum_form
    plan_t = Plan(dict(pr, kind=W.TABLE, spectrum_form=form), prec)
    plan_t.generate(table=torch.tensor(np.ascontiguousarray(tq), dtype=torch.float64, device="cuda"))
    assert plan_t.spectrum_form == form
    d, t = _products(torch, plan_t, m.reshape(shape_m), v.reshape(shape_v))
    assert rel_l2(d.reshape(nrhs, -1), m @ G.T) <= tol
    assert rel_l2(t.reshape(nrhs, -1), v @ G) <= tol
