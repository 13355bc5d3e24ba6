"""The products and the inversion driver captured in a HIP graph (through
torch.cuda.graph, which captures the library's launches on its stream):
every replay, with eager work and synchronisations between replays, equals
the eager call bit for bit.  The calls launch kernels only (no memsets, no
host synchronisation), which is what makes them capturable."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _capture(torch, fn):
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s):
        fn()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name", ["magnetic_48x56", "small_gravity"])
def test_cgls_replays_equal_eager(torch_cuda, name, prec):
    from paper_1912_06976_amd import Plan
    from paper_1912_06976_amd.plan import bttb_cgls, bttb_cgls_query
    torch = torch_cuda
    pr = getattr(W, name)()
    print("cgls graph", name, prec, flush=True)
    plan = Plan(pr, prec).generate()
    nx, ny, nz = W.dims(pr)
    d = torch.tensor(W.normal_data(pr, 7), dtype=plan.dtype, device="cuda").reshape(pr["sy"], pr["sx"])
    iters, lam = 12, 0.05
    ws = torch.empty(bttb_cgls_query(plan.handle), dtype=torch.uint8, device="cuda")
    m_ref = torch.zeros((nz, ny, nx), dtype=plan.dtype, device="cuda")
    h_ref = torch.zeros((iters + 1, 3), dtype=torch.float64, device="cuda")
    bttb_cgls(plan.handle, plan.spectra, d, m_ref, lam, iters, h_ref, ws)
    torch.cuda.synchronize()
    assert torch.isfinite(m_ref).all() and float(m_ref.abs().max()) > 0

    m = torch.zeros_like(m_ref)
    h = torch.zeros_like(h_ref)
    g = _capture(torch, lambda: bttb_cgls(plan.handle, plan.spectra, d, m, lam, iters, h, ws))
    other = torch.tensor(W.uniform_model(pr, 3), dtype=plan.dtype, device="cuda")
    for k in range(3):
        m.zero_()
        h.fill_(-1.0)
        plan.forward(other)            # eager work on the same spectra between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(m, m_ref), "replay %d" % k
        assert torch.equal(h, h_ref), "replay %d" % k


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_products_replay_equal_eager(torch_cuda, prec):
    from paper_1912_06976_amd import Plan
    from paper_1912_06976_amd.plan import bttb_forward, bttb_forward_noalloc, bttb_transpose
    torch = torch_cuda
    pr = W.magnetic_48x56()
    print("products graph", prec, flush=True)
    plan = Plan(pr, prec).generate()
    nx, ny, nz = W.dims(pr)
    nrhs = 2
    m = torch.tensor(W.uniform_model(pr, 11, nrhs=nrhs), dtype=plan.dtype, device="cuda")
    r = torch.tensor(W.normal_data(pr, 12, nrhs=nrhs), dtype=plan.dtype, device="cuda")
    ws = plan.workspace(nrhs)
    d_ref = plan.forward(m)
    mt_ref = plan.transpose(r)
    d_na_ref = torch.empty_like(d_ref)
    bttb_forward_noalloc(plan.handle, plan.spectra, m, d_na_ref, nrhs)   # first call sets up the array
    torch.cuda.synchronize()
    assert torch.equal(d_na_ref, d_ref)

    d = torch.empty_like(d_ref)
    mt = torch.empty_like(mt_ref)
    d_na = torch.empty_like(d_ref)

    def body():
        bttb_forward(plan.handle, plan.spectra, m, d, nrhs, ws)
        bttb_transpose(plan.handle, plan.spectra, r, mt, nrhs, ws)
        bttb_forward_noalloc(plan.handle, plan.spectra, m, d_na, nrhs)

    g = _capture(torch, body)
    m2 = torch.tensor(W.uniform_model(pr, 13, nrhs=nrhs), dtype=plan.dtype, device="cuda")
    for k in range(3):
        for t in (d, mt, d_na):
            t.fill_(float("nan"))
        plan.transpose(plan.forward(m2))   # eager products between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(d, d_ref), "replay %d" % k
        assert torch.equal(mt, mt_ref), "replay %d" % k
        assert torch.equal(d_na, d_ref), "replay %d" % k
    assert np.isfinite(d.double().cpu().numpy()).all()


def test_plan_methods_under_capture(torch_cuda):
    """Plan.forward / Plan.transpose inside a captured graph: outputs and the
    workspace come from the graph's memory pool (the workspace is not cached
    for later eager calls); replays and later eager calls on every stream
    equal the eager results bit for bit."""
    from paper_1912_06976_amd import Plan
    torch = torch_cuda
    pr = W.magnetic_48x56()
    plan = Plan(pr, "fp32").generate()
    m = torch.tensor(W.uniform_model(pr, 21), dtype=plan.dtype, device="cuda")
    r = torch.tensor(W.normal_data(pr, 22), dtype=plan.dtype, device="cuda")
    d_ref, mt_ref = plan.forward(m), plan.transpose(r)
    torch.cuda.synchronize()
    cached = dict(plan._ws)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s):
        d_g = plan.forward(m)
        mt_g = plan.transpose(r)
    torch.cuda.synchronize()
    # nothing of the graph's pool was cached
    assert set(plan._ws) == set(cached) and all(plan._ws[k] is cached[k] for k in cached)
    for k in range(3):
        plan.transpose(plan.forward(m))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(d_g, d_ref) and torch.equal(mt_g, mt_ref), "replay %d" % k
        with torch.cuda.stream(s):
            e = plan.forward(m)
        torch.cuda.synchronize()
        assert torch.equal(e, d_ref)
