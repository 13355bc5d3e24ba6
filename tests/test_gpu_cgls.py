"""The inversion driver (CGLS for min ||G m - d||^2 + lam^2 ||m||^2) against
the oracle's dense regularised solution, through the C ABI."""
import numpy as np
import pytest

import workloads as W
from _common import oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _case(pr, seed):
    import oracle
    P = oracle_problem(pr)
    G = oracle.dense_G_quad(P)
    rng = np.random.default_rng(seed)
    m_true = W.box_model(pr, seed, nboxes=2) if pr["kind"] == W.MAGNETIC else W.uniform_model(pr, seed)
    d = G @ m_true.ravel()
    d = d + 0.01 * np.std(d) * rng.standard_normal(d.shape)
    sv = np.linalg.svd(G, compute_uv=False)
    return G, d, sv


@pytest.mark.parametrize("name,prec,tol", [("small_gravity", "fp64", 1e-9), ("small_gravity", "fp32", 2e-4),
                                           ("magnetic_24", "fp64", 1e-9), ("magnetic_24", "fp32", 2e-4)])
def test_cgls_converges_to_dense_regularized_solution(torch_cuda, name, prec, tol):
    import oracle
    from paper_1912_06976_amd import Plan
    torch = torch_cuda
    pr = getattr(W, name)()
    print("cgls", name, prec, flush=True)
    G, d, sv = _case(pr, 61)
    lam = 0.1 * sv[0]
    ref = oracle.regularized_lsq(G, d, lam)
    plan = Plan(pr, prec).generate()
    dt = torch.tensor(d.reshape(pr["sy"], pr["sx"]), dtype=plan.dtype, device="cuda")
    m, hist = plan.cgls(dt, lam, 150)
    torch.cuda.synchronize()
    got = m.double().cpu().numpy().ravel()
    assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref), np.linalg.norm(got - ref) / np.linalg.norm(ref)
    h = hist.cpu().numpy()
    # start: r0 = d (m0 = 0), s0 = G^T d
    assert abs(h[0, 0] - d @ d) <= 1e-5 * (d @ d)
    gtd = G.T @ d
    assert abs(h[0, 2] - gtd @ gtd) <= 1e-5 * (gtd @ gtd)
    # the augmented residual ||r||^2 + lam^2 ||m||^2 never increases
    J = h[:, 0] + lam * lam * h[:, 1]
    slack = 1e-12 if prec == "fp64" else 1e-5
    assert np.all(np.diff(J) <= slack * J[0])
    # and ends at the minimum
    Jref = np.sum((G @ ref - d) ** 2) + lam * lam * ref @ ref
    assert abs(J[-1] - Jref) <= (1e-10 if prec == "fp64" else 1e-5) * Jref


@pytest.mark.parametrize("name,prec,tol", [("magnetic_24", "fp32", 2e-4), ("small_gravity", "fp32", 2e-4),
                                           ("magnetic_24", "fp64", 1e-9)])
def test_cgls_holds_the_solution_after_convergence(torch_cuda, name, prec, tol):
    """Many more steps than convergence needs: once ||s_k|| <= tau ||s_0||
    (tau = 1e-6 FP32, 1e-12 FP64) the steps leave m unchanged, so the
    iterate stays at the solution instead of drifting (in FP32 the products
    are each other's adjoint only to rounding); 150 and 600 steps then end
    on the same iterate, bit for bit, and the history repeats its last row."""
    import oracle
    from paper_1912_06976_amd import Plan
    torch = torch_cuda
    pr = getattr(W, name)()
    print("cgls long", name, prec, flush=True)
    G, d, sv = _case(pr, 61)
    lam = 0.1 * sv[0]
    ref = oracle.regularized_lsq(G, d, lam)
    plan = Plan(pr, prec).generate()
    dt = torch.tensor(d.reshape(pr["sy"], pr["sx"]), dtype=plan.dtype, device="cuda")
    tau = 1e-6 if prec == "fp32" else 1e-12
    m150, _ = plan.cgls(dt, lam, 150)
    m600, h = plan.cgls(dt, lam, 600)
    torch.cuda.synchronize()
    h = h.cpu().numpy()
    stop = int(np.argmax(h[:, 2] <= tau * tau * h[0, 2]))
    assert h[stop, 2] <= tau * tau * h[0, 2] and 0 < stop < 150, stop
    assert np.array_equal(h[stop:], np.broadcast_to(h[stop], h[stop:].shape))
    assert torch.equal(m150, m600)
    got = m600.double().cpu().numpy().ravel()
    assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref), np.linalg.norm(got - ref) / np.linalg.norm(ref)


def test_cgls_warm_start_zero_steps_and_validation(torch_cuda):
    import paper_1912_06976_amd as B
    from paper_1912_06976_amd import Plan
    torch = torch_cuda
    pr = W.small_gravity()
    G, d, sv = _case(pr, 62)
    plan = Plan(pr, "fp64").generate()
    dt = torch.tensor(d.reshape(pr["sy"], pr["sx"]), dtype=torch.float64, device="cuda")
    m0 = torch.tensor(W.normal_model(pr, 63), dtype=torch.float64, device="cuda")
    m, hist = plan.cgls(dt, 0.2 * sv[0], 0, m0=m0)
    torch.cuda.synchronize()
    assert torch.equal(m, m0)
    r0 = d - G @ m0.cpu().numpy().ravel()
    assert abs(hist[0, 0].item() - r0 @ r0) <= 1e-10 * (r0 @ r0)
    # a warm start continues the same minimisation
    lam = 0.2 * sv[0]
    m1, _ = plan.cgls(dt, lam, 8)
    m2, _ = plan.cgls(dt, lam, 8, m0=m1)
    import oracle
    ref = oracle.regularized_lsq(G, d, lam)
    e1 = np.linalg.norm(m1.cpu().numpy().ravel() - ref)
    e2 = np.linalg.norm(m2.cpu().numpy().ravel() - ref)
    assert e2 <= 0.5 * e1
    ws = torch.empty(B.bttb_cgls_query(plan.handle), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.BttbError):
        B.bttb_cgls(plan.handle, plan.spectra, dt, m1, -1.0, 5, None, ws)
    with pytest.raises(B.BttbError):
        B.bttb_cgls(plan.handle, plan.spectra, dt, m1, 1.0, 5, None, ws[:-256])
