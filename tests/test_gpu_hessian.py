"""User-chosen kernels evaluated on the device (Sec. 1 (vi)): "hessian"
plans, sum_ab w_ab U_ab of the second derivatives of the prism potential with
respect to the station, generated from the closed forms on the GPU (the
Laplace-eliminated five-term corner function), against the oracle's dense
matrix (each component from its own closed form, U_zz directly).

Kernels: the total-field anomaly of a remanent magnetisation (field and
magnetisation directions differ), the gravity gradient g_zz (even in both
offsets: real even spectra by default, and the complex form), the vertical
field B_z of a magnetisation, and seeded random weights; FP64 and FP32; h = 0
(air-side values on the top faces) and raised stations; one shape at
12-point transform lengths.  Generated entries are held to the FP64 bar of
_common.fp64_bar, the exact entries supplied as a table to 1e-12, FP32 to
2e-5 (rel-L2 per right-hand side, Sec. 5)."""
import math

import numpy as np
import pytest

import workloads as W
from _common import fp64_bar, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5}


def _dir(incl, decl):
    i, d = math.radians(incl), math.radians(decl)
    return (math.cos(i) * math.cos(d), math.cos(i) * math.sin(d), math.sin(i))


def _sym(f, m):
    return (f[0] * m[0], f[1] * m[1], f[2] * m[2], f[0] * m[1] + f[1] * m[0], f[0] * m[2] + f[2] * m[0],
            f[1] * m[2] + f[2] * m[1])


_RNG = np.random.default_rng(7300)
CASES = {
    # remanent magnetisation: field (60, 15), magnetisation (-30, 100), 100 nT per A/m
    "remanent_tmi": W.problem(W.HESSIAN, 20, 24, 5, 3, 2, 4, 1, dx=100.0, dy=100.0, dz=50.0, scale=100.0,
                              hessian=_sym(_dir(60.0, 15.0), _dir(-30.0, 100.0))),
    # g_zz in Eotvos per g/cm^3, raised stations
    "gzz_even": dict(W.problem(W.HESSIAN, 18, 15, 4, 2, 2, 3, 3, dx=50.0, dy=50.0, dz=25.0, h=10.0,
                               scale=66.743, hessian=(0, 0, 1, 0, 0, 0)), spectrum_form="auto"),
    "gzz_complex": dict(W.problem(W.HESSIAN, 18, 15, 4, 2, 2, 3, 3, dx=50.0, dy=50.0, dz=25.0, h=10.0,
                                  scale=66.743, hessian=(0, 0, 1, 0, 0, 0)), spectrum_form="complex"),
    # g_xx + g_yy with asymmetric padding at h = 0 (real even form)
    "gxx_gyy_h0": W.problem(W.HESSIAN, 16, 13, 3, 4, 1, 0, 2, dx=25.0, dy=50.0, dz=25.0, scale=66.743,
                            hessian=(1, 1, 0, 0, 0, 0)),
    # vertical field of a magnetisation m: B_z = sum_b U_zb m_b
    "bz": W.problem(W.HESSIAN, 22, 17, 4, 2, 3, 1, 2, dx=100.0, dy=100.0, dz=50.0, h=5.0, scale=100.0,
                    hessian=(0.0, 0.0, _dir(45.0, 30.0)[2], 0.0, _dir(45.0, 30.0)[0], _dir(45.0, 30.0)[1])),
    "random": W.problem(W.HESSIAN, 19, 21, 3, 1, 4, 2, 0, dx=50.0, dy=100.0, dz=50.0,
                        hessian=tuple(_RNG.uniform(-1.0, 1.0, size=6))),
    # 12-point lengths along both axes (96 x 144)
    "remanent_mixed": W.problem(W.HESSIAN, 40, 60, 3, 9, 8, 12, 10, dx=100.0, dy=100.0, dz=50.0, scale=100.0,
                                hessian=_sym(_dir(70.0, -20.0), _dir(10.0, 160.0))),
}
FORMS = {"remanent_tmi": "complex", "gzz_even": "real_even", "gzz_complex": "complex", "gxx_gyy_h0": "real_even",
         "bz": "complex", "random": "complex", "remanent_mixed": "complex"}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


_CACHE = {}


def _oracle(name):
    import oracle
    if name not in _CACHE:
        P = oracle_problem(CASES[name])
        _CACHE.clear()
        _CACHE[name] = (oracle.dense_G_quad(P), oracle.dense_G(P), oracle.offset_table_quad(P)[0])
    return _CACHE[name]


def _products(torch, plan, m, v):
    d = plan.forward(torch.tensor(m, dtype=plan.dtype, device="cuda"))
    t = plan.transpose(torch.tensor(v, dtype=plan.dtype, device="cuda"))
    torch.cuda.synchronize()
    return d.double().cpu().numpy().reshape(m.shape[0], -1), t.double().cpu().numpy().reshape(v.shape[0], -1)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_hessian_kernel_parity(torch_cuda, name, prec):
    from paper_1912_06976_amd import Plan
    torch = torch_cuda
    pr = CASES[name]
    print("hessian", name, prec, flush=True)
    G, Gp, tq = _oracle(name)
    nrhs = 2
    m = W.normal_model(pr, 7100, nrhs=nrhs)
    v = W.normal_data(pr, 7200, nrhs=nrhs)
    mf, vf = m.reshape(nrhs, -1), v.reshape(nrhs, -1)
    tol = TOL[prec]
    plan = Plan(pr, prec).generate()
    assert plan.spectrum_form == FORMS[name]
    d, t = _products(torch, plan, m, v)
    for q in range(nrhs):
        bf = fp64_bar(Gp, G, mf[q]) if prec == "fp64" else tol
        bt = fp64_bar(Gp, G, vf[q], transpose=True) if prec == "fp64" else tol
        assert rel_l2(d[q], G @ mf[q]) <= bf, ("forward", q)
        assert rel_l2(t[q], G.T @ vf[q]) <= bt, ("transpose", q)
    form = plan.spectrum_form
    del plan
    # the exact entries through the table route: the stated bar
    plan_t = Plan(dict(pr, kind=W.TABLE, spectrum_form=form, scale=1.0), prec)
    plan_t.generate(table=torch.tensor(np.ascontiguousarray(tq), dtype=torch.float64, device="cuda"))
    d, t = _products(torch, plan_t, m, v)
    assert rel_l2(d, mf @ G.T) <= tol
    assert rel_l2(t, vf @ G) <= tol


def test_induced_weights_equal_the_magnetic_kernel(torch_cuda):
    # w = f f^T with scale F / (4 pi) is the induced kernel of Sec. 4.2: the
    # same corner function and weights on the device, so the same spectra
    from paper_1912_06976_amd import Plan
    torch = torch_cuda
    mag = W.magnetic_48x56()
    f = _dir(mag["incl"], mag["decl"])
    hes = dict(mag, kind=W.HESSIAN, hessian=_sym(f, f), scale=mag["field_nT"] / (4 * math.pi))
    m = torch.tensor(W.normal_model(mag, 7300), dtype=torch.float64, device="cuda")
    a = Plan(mag, "fp64").generate().forward(m)
    b = Plan(hes, "fp64").generate().forward(m)
    torch.cuda.synchronize()
    assert rel_l2(b.cpu().numpy().ravel(), a.cpu().numpy().ravel()) <= 1e-14
