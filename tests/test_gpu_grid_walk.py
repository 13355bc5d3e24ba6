"""The persistent kernels (row transforms, transpose multiply-accumulate) size
their grids to the blocks resident at once and walk the work units: a block
decodes its first unit and advances the position from there (row groups by
the grid size, transpose units one by one), decoding again where the walk
enters the next job.  With the grid capped (bttb_debug_cap_grid) every block
walks many units, across batch and job boundaries and with every remainder
of the step; each unit is computed on its own, so the products must equal
the uncapped ones bit for bit."""
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CAPS = (1, 3, 7, 61)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture
def capped():
    from paper_1912_06976_amd import bttb_debug_cap_grid
    yield bttb_debug_cap_grid
    bttb_debug_cap_grid(0)


def _shapes():
    odd = W.problem(W.GRAVITY, 29, 37, 5, 2, 3, 1, 2, dx=40.0, dy=30.0, dz=20.0)
    tile8 = dict(W.magnetic_48x56(), row_tile=8)
    mixed = W.problem(W.MAGNETIC, 60, 50, 6, 3, 4, 2, 2, dx=50.0, dy=50.0, dz=25.0,
                      incl=55.0, decl=10.0, nx_fft=144, ny_fft=192)
    return {"small_gravity": W.small_gravity(), "magnetic_48x56": W.magnetic_48x56(),
            "odd_rows": odd, "row_tile_8": tile8, "lengths_144x192": mixed}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name", sorted(_shapes()))
def test_capped_grid_equals_default(torch_cuda, capped, name, prec):
    from paper_1912_06976_amd import Plan
    torch = torch_cuda
    pr = _shapes()[name]
    print("grid walk", name, prec, flush=True)
    plan = Plan(pr, prec).generate()
    nrhs = 3
    m = torch.tensor(W.uniform_model(pr, 31, nrhs=nrhs), dtype=plan.dtype, device="cuda")
    r = torch.tensor(W.normal_data(pr, 32, nrhs=nrhs), dtype=plan.dtype, device="cuda")
    d_ref, mt_ref = plan.forward(m), plan.transpose(r)
    torch.cuda.synchronize()
    assert torch.isfinite(d_ref).all() and torch.isfinite(mt_ref).all()
    for cap in CAPS:
        capped(cap)
        d, mt = plan.forward(m), plan.transpose(r)
        torch.cuda.synchronize()
        assert torch.equal(d, d_ref), "forward, cap %d" % cap
        assert torch.equal(mt, mt_ref), "transpose, cap %d" % cap
    capped(0)
    assert torch.equal(plan.forward(m), d_ref)


def test_capped_grid_batch(torch_cuda, capped):
    """Multi-job launches: the first twelve instances of the 48-instance batch
    (several instances per launch, 2^a 3^b and power-of-two lengths, both
    spectrum forms), captured once with the default grids and once with a
    capped grid."""
    from paper_1912_06976_amd import Batch, Plan
    torch = torch_cuda
    probs = W.batch48()[:12]
    plans = [Plan(p, "fp32").generate() for p in probs]
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    ms = [torch.randn((2, p.nz, p.ny, p.nx), generator=g, device="cuda") for p in plans]
    rs = [torch.randn((2, p.sy, p.sx), generator=g, device="cuda") for p in plans]
    ds_ref, mts_ref = Batch(plans, max_nrhs=2).run(ms, rs)
    torch.cuda.synchronize()
    for cap in (5, 29):
        capped(cap)
        ds, mts = Batch(plans, max_nrhs=2).run(ms, rs)   # captured with the cap
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert torch.equal(ds[i], ds_ref[i]), "forward %d, cap %d" % (i, cap)
            assert torch.equal(mts[i], mts_ref[i]), "transpose %d, cap %d" % (i, cap)
