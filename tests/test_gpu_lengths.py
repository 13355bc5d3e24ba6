"""Every power-of-two transform length the workloads use (256, 512, 1024)
along x and along y, against the oracle's dense matrix.

For each length and axis three shapes are taken (the other axis is short):
  wide    3 stations and wide padding: the model extends past half the
          transform (the forward's first stage is not pruned)
  half    stations over nearly half the transform, the model just past half
  pruned  a small volume with the length requested explicitly (pruned first
          stages)
each for gravity in the real even and in the complex spectrum form and for the
magnetic kernel, in FP64 and FP32.  Generated entries are held to the FP64 bar
of _common.fp64_bar; the exact entries supplied as a table to 1e-12 (FP64);
FP32 to 2e-5 (Sec. 5 error metric, rel-L2 per right-hand side).
"""
import numpy as np
import pytest

import workloads as W
from _common import fp64_bar, oracle_problem, rel_l2

TOL = {"fp64": 1e-12, "fp32": 2e-5}
LENGTHS = (256, 512, 1024)
VARIANTS = ("wide", "half", "pruned")
KINDS = ("gravity_even", "gravity_complex", "magnetic")


def shape(axis, N, variant, kind):
    """Problem whose transform along `axis` has length N (the other axis: 2
    stations, length 8)."""
    mag = kind == "magnetic"
    if variant == "wide":
        P = (N - 5) // 2 - 2                   # s + n - 1 = 2 P + 5 <= N, n = 2 P + 3 > N / 2
        s, pl, pr_ = 3, P, P
        if mag:
            pl, pr_ = P - 5, P + 5
        nfft = 0
    elif variant == "half":
        s, pl, pr_ = N // 2 - 40, 20, 25      # n = N / 2 + 5, s + n - 1 = N - 36
        if mag:
            pl, pr_ = 25, 20
        nfft = 0
    else:
        s, pl, pr_ = 20, 3, 4
        nfft = N
    o_s, o_l, o_r = 2, 1, (0 if mag else 1)
    kw = dict(dx=25.0, dy=50.0, dz=20.0, h=2.5 if variant == "half" else 0.0)
    if mag:
        kw.update(incl=55.0, decl=-35.0, field_nT=47000.0)
    k = W.MAGNETIC if mag else W.GRAVITY
    if axis == "x":
        pr = W.problem(k, s, o_s, 2, pl, pr_, o_l, o_r, nx_fft=nfft, **kw)
    else:
        pr = W.problem(k, o_s, s, 2, o_l, o_r, pl, pr_, ny_fft=nfft, **kw)
    pr["spectrum_form"] = "complex" if kind == "gravity_complex" else "auto"
    return pr


def test_shapes_reach_their_lengths_and_pruning():
    # host-side check of the shape recipe (no GPU): each shape's minimal
    # power-of-two length is N, and "wide"/"half" put the model past N / 2
    for axis in ("x", "y"):
        for N in LENGTHS:
            for variant in VARIANTS:
                for kind in KINDS:
                    pr = shape(axis, N, variant, kind)
                    nx, ny, _ = W.dims(pr)
                    s, n = (pr["sx"], nx) if axis == "x" else (pr["sy"], ny)
                    req = pr["nx_fft"] if axis == "x" else pr["ny_fft"]
                    if req:
                        assert req == N and n <= N // 2
                    else:
                        assert N // 2 < s + n - 1 <= N and n > N // 2
                        if kind == "gravity_even":
                            pl, prr = (pr["pxl"], pr["pxr"]) if axis == "x" else (pr["pyl"], pr["pyr"])
                            assert 2 * (s - 1 + max(pl, prr)) + 1 <= N


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


_CACHE = {}


def _oracle(pr):
    import oracle
    key = repr(sorted((k, str(v)) for k, v in pr.items() if k != "spectrum_form"))
    if key not in _CACHE:
        P = oracle_problem(pr)
        _CACHE.clear()
        _CACHE[key] = (oracle.dense_G_quad(P), oracle.dense_G(P), oracle.offset_table_quad(P)[0])
    return _CACHE[key]


def _products(torch, plan, m, v):
    d = plan.forward(torch.tensor(m, dtype=plan.dtype, device="cuda"))
    t = plan.transpose(torch.tensor(v, dtype=plan.dtype, device="cuda"))
    torch.cuda.synchronize()
    return d.double().cpu().numpy().reshape(m.shape[0], -1), t.double().cpu().numpy().reshape(v.shape[0], -1)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("N", LENGTHS)
@pytest.mark.parametrize("axis", ["x", "y"])
def test_length_parity(torch_cuda, axis, N, variant, kind, prec):
    from paper_1912_06976_amd import Plan
    torch = torch_cuda
    pr = shape(axis, N, variant, kind)
    print("length", axis, N, variant, kind, prec, flush=True)
    G, Gp, tq = _oracle(pr)
    nrhs = 2
    m = W.normal_model(pr, 5100 + N, nrhs=nrhs)
    v = W.normal_data(pr, 5200 + N, nrhs=nrhs)
    mf, vf = m.reshape(nrhs, -1), v.reshape(nrhs, -1)
    tol = TOL[prec]

    plan = Plan(pr, prec).generate()
    assert (plan.nx_fft if axis == "x" else plan.ny_fft) == N
    assert plan.spectrum_form == ("real_even" if kind == "gravity_even" else "complex")
    d, t = _products(torch, plan, m, v)
    for q in range(nrhs):
        bf = fp64_bar(Gp, G, mf[q]) if prec == "fp64" else tol
        bt = fp64_bar(Gp, G, vf[q], transpose=True) if prec == "fp64" else tol
        assert rel_l2(d[q], G @ mf[q]) <= bf, ("forward", q)
        assert rel_l2(t[q], G.T @ vf[q]) <= bt, ("transpose", q)
    form = plan.spectrum_form
    del plan

    # the exact entries as a table: the stated bar
    plan_t = Plan(dict(pr, kind=W.TABLE, spectrum_form=form), prec)
    plan_t.generate(table=torch.tensor(np.ascontiguousarray(tq), dtype=torch.float64, device="cuda"))
    d, t = _products(torch, plan_t, m, v)
    assert rel_l2(d, mf @ G.T) <= tol
    assert rel_l2(t, vf @ G) <= tol
