"""The forward product without a workspace argument (bttb_forward_noalloc,
for callers that cannot allocate): called through the C ABI on several calls
in a row, each with a smaller input than the one before, its output must
equal bttb_forward's with a caller workspace, bit for bit (same kernels, same
workspace layout, same depth split)."""
import numpy as np
import pytest

import workloads as W
from _common import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _both(torch, plan, nrhs, seed):
    import paper_1912_06976_amd as B
    m = torch.tensor(W.normal_model(plan.problem, seed, nrhs), dtype=plan.dtype, device="cuda")
    ref = torch.empty((nrhs, plan.sy, plan.sx), dtype=plan.dtype, device="cuda")
    got = torch.full((nrhs, plan.sy, plan.sx), float("nan"), dtype=plan.dtype, device="cuda")
    ws = torch.empty(plan.workspace_bytes(nrhs), dtype=torch.uint8, device="cuda")
    B.bttb_forward(plan.handle, plan.spectra, m, ref, nrhs, ws)
    torch.cuda.synchronize()
    B.bttb_forward_noalloc(plan.handle, plan.spectra, m, got, nrhs)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-5), ("fp64", 1e-12)])
def test_noalloc_forward_equals_forward_on_shrinking_calls(torch_cuda, prec, tol):
    from paper_1912_06976_amd import Plan
    big = Plan(W.magnetic_48x56(), prec).generate()
    small = Plan(W.small_gravity(), prec).generate()
    torch_cuda.cuda.synchronize()
    # (plan, nrhs): every call's input is smaller than the previous one's;
    # both plans split the depth sum (partial sums in the scratch array)
    calls = [(big, 3), (big, 1), (small, 2), (small, 1)]
    for k, (plan, nrhs) in enumerate(calls):
        print("noalloc call", k, prec, plan.problem["kind"], plan.nz, "nrhs", nrhs, flush=True)
        assert plan.workspace_bytes(nrhs) <= 64 << 20
        ref, got = _both(torch_cuda, plan, nrhs, 900 + k)
        assert np.all(np.isfinite(got))
        assert rel_l2(got, ref) <= tol
        assert np.array_equal(got, ref)
