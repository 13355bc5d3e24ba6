"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: index maps bit-exact; FP64 products rel-L2 <= 1e-12 against the
oracle's dense G with entries evaluated in __float128 (for entries generated
in FP64 from the closed forms: the larger of 1e-12 and 10x the oracle's own
plain-FP64 error on the same product, see _common.fp64_bar); FP32 products
rel-L2 <= 2e-5; generator entries within 32 eps of the size of their
cancelling corner terms.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from _common import fp64_bar, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 2e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def _plan(pr, prec, acc="default"):
    from paper_1912_06976_amd import Plan
    return Plan(pr, prec, acc).generate()


def _dense_ref(orc, pr):
    P = oracle_problem(pr)
    return P, orc.dense_G_quad(P)


# ---------------------------------------------------------------------------
# generator
# ---------------------------------------------------------------------------

PROBE_SHAPES = [
    W.problem(W.PROBE, 5, 4, 3, 2, 1, 1, 2, dx=25.0, dy=50.0, dz=10.0),
    W.problem(W.PROBE, 7, 3, 2, 0, 4, 3, 0, dx=10.0, dy=10.0, dz=10.0, nx_fft=32, ny_fft=16),
    W.problem(W.PROBE, 1, 1, 1, 0, 0, 0, 0, dx=1.0, dy=1.0, dz=1.0),
    W.problem(W.PROBE, 12, 9, 2, 3, 3, 0, 2, dx=5.0, dy=5.0, dz=5.0),
]


@pytest.mark.parametrize("k", range(len(PROBE_SHAPES)))
def test_probe_generator_reproduces_dense_matrix(torch_cuda, orc, k):
    pr = PROBE_SHAPES[k]
    _say("probe generator", pr["sx"], pr["sy"], pr["nz"])
    P = oracle_problem(pr)
    G = orc.dense_G(P)
    from paper_1912_06976_amd import Plan
    plan = Plan(pr, "fp64")
    Nx, Ny = plan.nx_fft, plan.ny_fft
    for r in range(P.nz):
        T = plan.debug_generator(r)
        assert T.shape == (Ny, Nx)
        covered = np.zeros((Ny, Nx), dtype=bool)
        for j in range(P.sy):
            for i in range(P.sx):
                for q in range(P.ny):
                    for p in range(P.nx):
                        a = ((j - q) % Ny, (i - p) % Nx)
                        assert T[a] == G[j * P.sx + i, r * P.nx * P.ny + q * P.nx + p]
                        covered[a] = True
        assert np.all(T[~covered] == 0.0)


def test_paper_circulant_example(torch_cuda):
    # Sec. 3: the 3 x 3 Toeplitz matrix with first row (g1, g2, g3) and first
    # column (g1, gamma2, gamma3) embeds in the circulant with first column
    # (g1, gamma2, gamma3, g3, g2); with a longer transform zeros fill the gap
    ex = None
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_index_examples.txt")):
        if line.startswith("column"):
            ex = line.split()[1:]
    assert ex == ["g1", "gamma2", "gamma3", "g3", "g2"]
    from paper_1912_06976_amd import Plan
    plan = Plan(W.problem(W.PROBE, 3, 1, 1, dx=1.0, dy=1.0, dz=1.0), "fp64")
    col = plan.debug_generator(0)[0]            # y offset 0 row, x varies
    lab = {0: "g1", -1: "gamma2", -2: "gamma3", 2: "g3", 1: "g2"}
    nz = [lab[int(v)] for v in np.concatenate([col[:3], col[-2:]])]
    assert nz == ex
    assert np.all(col[3:-2] == 0)


@pytest.mark.parametrize("pr", [W.small_gravity(), dict(W.small_gravity(), spectrum_form="complex"),
                                W.problem(W.GRAVITY, 10, 7, 2, 2, 5, 1, 0, dx=30.0, dy=30.0, dz=15.0, h=3.0,
                                          nx_fft=64, ny_fft=32),
                                W.magnetic_48x56(),
                                W.problem(W.MAGNETIC, 9, 6, 3, 1, 2, 2, 1, dx=50.0, dy=100.0, dz=30.0,
                                          h=7.0, incl=-30.0, decl=140.0, field_nT=52000.0)])
def test_generator_entries_match_quad_oracle(torch_cuda, orc, pr):
    _say("generator entries", pr["kind"], pr["sx"], pr["sy"])
    P = oracle_problem(pr)
    t, a = orc.offset_table_quad(P)      # [nz][wy][wx], index = offset + (s - 1 + pl)
    from paper_1912_06976_amd import Plan
    plan = Plan(pr, "fp64")
    Nx, Ny = plan.nx_fft, plan.ny_fft
    eps = np.finfo(float).eps
    for r in range(P.nz):
        T = plan.debug_generator(r)
        if plan.spectrum_form == "complex":
            # T[ay mod Ny][ax mod Nx] = h(-ax - pxl, -ay - pyl) for ax in [-(nx-1), sx-1]
            ax = np.arange(-(P.nx - 1), P.sx)
            ay = np.arange(-(P.ny - 1), P.sy)
            ox = -ax - P.pxl
            oy = -ay - P.pyl
        else:
            # centred even placement: T[ay mod Ny][ax mod Nx] = h(|ax|, |ay|) for
            # |ax| <= sx - 1 + max(pxl, pxr) (h is even: take the offset sign
            # the oracle's table covers)
            bx, by = P.sx - 1 + max(P.pxl, P.pxr), P.sy - 1 + max(P.pyl, P.pyr)
            ax = np.arange(-bx, bx + 1)
            ay = np.arange(-by, by + 1)
            ox = np.where(np.abs(ax) <= P.nx - 1 - P.pxl, np.abs(ax), -np.abs(ax))
            oy = np.where(np.abs(ay) <= P.ny - 1 - P.pyl, np.abs(ay), -np.abs(ay))
        got = T[np.ix_(ay % Ny, ax % Nx)]
        ix = ox + (P.sx - 1 + P.pxl)
        iy = oy + (P.sy - 1 + P.pyl)
        ref = t[r][np.ix_(iy, ix)]
        bound = 32 * eps * a[r][np.ix_(iy, ix)] + 1e-300
        assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)
        rest = np.ones((Ny, Nx), dtype=bool)
        rest[np.ix_(ay % Ny, ax % Nx)] = False
        assert np.all(T[rest] == 0.0)


# ---------------------------------------------------------------------------
# products against the dense oracle
# ---------------------------------------------------------------------------

def _products(torch, plan, m, v):
    dt = plan.dtype
    mt = torch.tensor(m, dtype=dt, device="cuda")
    vt = torch.tensor(v, dtype=dt, device="cuda")
    d = plan.forward(mt)
    t = plan.transpose(vt)
    torch.cuda.synchronize()
    return d.double().cpu().numpy(), t.double().cpu().numpy()


@pytest.mark.parametrize("form", ["auto", "complex"])
def test_small_gravity_fp64(torch_cuda, orc, form):
    pr = dict(W.small_gravity(), spectrum_form=form)
    _say("small gravity fp64", form)
    P, G = _dense_ref(orc, pr)
    m = W.uniform_model(pr, 101)
    v = W.normal_data(pr, 102)
    d, t = _products(torch_cuda, _plan(pr, "fp64"), m, v)
    assert rel_l2(d.ravel(), G @ m.ravel()) <= TOL64
    assert rel_l2(t.ravel(), G.T @ v.ravel()) <= TOL64


@pytest.fixture(scope="module")
def magnetic_case(orc):
    pr = W.magnetic_48x56()
    P, G = _dense_ref(orc, pr)
    m = W.box_model(pr, 201, nboxes=3, noise_std=1e-4)
    v = W.normal_data(pr, 202)
    return pr, G, m, v


def test_magnetic_fp64(torch_cuda, magnetic_case):
    pr, G, m, v = magnetic_case
    _say("magnetic 48x56 fp64")
    d, t = _products(torch_cuda, _plan(pr, "fp64"), m, v)
    assert rel_l2(d.ravel(), G @ m.ravel()) <= TOL64
    assert rel_l2(t.ravel(), G.T @ v.ravel()) <= TOL64


@pytest.mark.parametrize("acc", ["default", "plain", "twosum", "wide"])
def test_magnetic_fp32(torch_cuda, magnetic_case, acc):
    pr, G, m, v = magnetic_case
    _say("magnetic 48x56 fp32", acc)
    d, t = _products(torch_cuda, _plan(pr, "fp32", acc), m, v)
    assert rel_l2(d.ravel(), G @ m.ravel()) <= TOL32
    assert rel_l2(t.ravel(), G.T @ v.ravel()) <= TOL32


EDGE = [
    W.problem(W.GRAVITY, 1, 1, 1, dx=10.0, dy=10.0, dz=10.0),
    W.problem(W.GRAVITY, 1, 6, 2, 0, 0, 2, 1, dx=10.0, dy=20.0, dz=5.0),
    W.problem(W.MAGNETIC, 7, 1, 3, 3, 0, 0, 0, dx=50.0, dy=50.0, dz=25.0, incl=70.0, decl=-20.0,
              field_nT=48000.0),
    W.problem(W.MAGNETIC, 13, 11, 5, 0, 3, 4, 1, dx=25.0, dy=40.0, z_edges=[0, 10, 25, 45, 70, 100],
              h=12.5, incl=35.0, decl=70.0, field_nT=45000.0),
    W.problem(W.GRAVITY, 10, 7, 4, 2, 5, 1, 0, dx=30.0, dy=30.0, dz=15.0, h=3.0, nx_fft=64, ny_fft=32),
    W.problem(W.MAGNETIC, 33, 30, 3, 1, 1, 1, 1, dx=100.0, dy=100.0, dz=50.0, incl=-60.0, decl=5.0,
              field_nT=47000.0),
    W.problem(W.GRAVITY, 70, 9, 2, 3, 2, 0, 0, dx=25.0, dy=25.0, dz=20.0),  # Nx = 128, Ny = 16
]


@pytest.mark.parametrize("k", range(len(EDGE)))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("row_tile", [4, 8])
@pytest.mark.parametrize("form", ["auto", "complex"])
def test_edge_shapes(torch_cuda, orc, k, prec, row_tile, form):
    if form == "complex" and EDGE[k]["kind"] != W.GRAVITY:
        pytest.skip("the complex form is the only one for this kernel (covered by 'auto')")
    pr = dict(EDGE[k], row_tile=row_tile, spectrum_form=form)
    _say("edge shape", k, prec, row_tile, form)
    P, G = _dense_ref(orc, pr)
    m = W.normal_model(pr, 1000 + k)
    v = W.normal_data(pr, 2000 + k)
    d, t = _products(torch_cuda, _plan(pr, prec), m, v)
    tol = TOL64 if prec == "fp64" else TOL32
    assert rel_l2(d.ravel(), G @ m.ravel()) <= tol
    assert rel_l2(t.ravel(), G.T @ v.ravel()) <= tol


@pytest.mark.parametrize("acc", ["default", "plain", "twosum", "wide"])
@pytest.mark.parametrize("form", ["auto", "complex"])
def test_gravity_fp32_odd_padding(torch_cuda, orc, acc, form):
    # odd left padding in x and y (phase sign at the Nyquist column), a
    # uniform model as in the paper's gravity experiments
    pr = dict(W.problem(W.GRAVITY, 23, 17, 6, 3, 2, 5, 4, dx=40.0, dy=25.0, dz=20.0, h=5.0), spectrum_form=form)
    _say("gravity fp32 odd padding", acc, form)
    P, G = _dense_ref(orc, pr)
    m = W.uniform_model(pr, 121)
    v = W.normal_data(pr, 122)
    plan = _plan(pr, "fp32", acc)
    assert plan.spectrum_form == ("real_even" if form == "auto" else "complex")
    d, t = _products(torch_cuda, plan, m, v)
    assert rel_l2(d.ravel(), G @ m.ravel()) <= TOL32
    assert rel_l2(t.ravel(), G.T @ v.ravel()) <= TOL32


@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("kind", [W.GRAVITY, W.MAGNETIC])
def test_table1_padded_shapes_fp64(torch_cuda, orc, k, kind):
    kw = dict(dx=50.0, dy=50.0, dz=25.0)
    if kind == W.MAGNETIC:
        kw.update(incl=60.0, decl=15.0, field_nT=47000.0)
    pr = W.table1_problem(k, kind, padded=True, **kw)
    _say("table1", k, kind)
    P = oracle_problem(pr)
    G = orc.dense_G_quad(P)
    Gp = orc.dense_G(P)
    m = W.normal_model(pr, 300 + k)
    v = W.normal_data(pr, 400 + k)
    plan = _plan(pr, "fp64")
    d, t = _products(torch_cuda, plan, m, v)
    # Entries generated in FP64 from the closed-form corner sums carry the
    # rounding of their cancelling terms for distant prisms; the bar is the
    # larger of 1e-12 and 10x the error the oracle's own plain-FP64 entries
    # make on the same product (fp64_bar)
    assert rel_l2(d.ravel(), G @ m.ravel()) <= fp64_bar(Gp, G, m)
    assert rel_l2(t.ravel(), G.T @ v.ravel()) <= fp64_bar(Gp, G, v, transpose=True)
    # the exact entries supplied as a table: the stated bar, 1e-12
    import torch
    tq, _ = orc.offset_table_quad(P)
    from paper_1912_06976_amd import Plan
    plan_t = Plan(dict(pr, kind=W.TABLE, spectrum_form=plan.spectrum_form), "fp64")
    plan_t.generate(table=torch.tensor(np.ascontiguousarray(tq), dtype=torch.float64, device="cuda"))
    d, t = _products(torch_cuda, plan_t, m, v)
    assert rel_l2(d.ravel(), G @ m.ravel()) <= TOL64
    assert rel_l2(t.ravel(), G.T @ v.ravel()) <= TOL64


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multiple_rhs_equal_single(torch_cuda, orc, prec):
    torch = torch_cuda
    pr = EDGE[3]
    plan = _plan(pr, prec)
    m = W.normal_model(pr, 55, nrhs=3)
    v = W.normal_data(pr, 56, nrhs=3)
    d3, t3 = _products(torch, plan, m, v)
    P, G = _dense_ref(orc, pr)
    tol = TOL64 if prec == "fp64" else TOL32
    assert rel_l2(d3.reshape(3, -1), m.reshape(3, -1) @ G.T) <= tol
    assert rel_l2(t3.reshape(3, -1), v.reshape(3, -1) @ G) <= tol
    for q in range(3):
        d1, t1 = _products(torch, plan, m[q], v[q])
        assert np.array_equal(d1, d3[q]) and np.array_equal(t1, t3[q])


@pytest.mark.parametrize("chunk", [1, 2, 3])
def test_layer_chunked_transpose_equals_unchunked(torch_cuda, orc, chunk):
    torch = torch_cuda
    pr = EDGE[3]                       # 5 layers: chunks of 1, 2 (ragged) and 3 (ragged)
    a = _plan(pr, "fp32")
    b = _plan(dict(pr, layer_chunk=chunk), "fp32")
    v = W.normal_data(pr, 66, nrhs=2)
    _, ta = _products(torch, a, W.normal_model(pr, 65, nrhs=2), v)
    _, tb = _products(torch, b, W.normal_model(pr, 65, nrhs=2), v)
    assert np.array_equal(ta, tb)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-5)])
def test_adjoint_identity(torch_cuda, prec, tol):
    pr = W.magnetic_24()
    plan = _plan(pr, prec)
    m = W.normal_model(pr, 77)
    v = W.normal_data(pr, 78)
    d, t = _products(torch_cuda, plan, m, v)
    lhs, rhs = float(d.ravel() @ v.ravel()), float(m.ravel() @ t.ravel())
    assert abs(lhs - rhs) <= tol * np.linalg.norm(d) * np.linalg.norm(v)


def test_deterministic(torch_cuda):
    pr = W.magnetic_48x56()
    plan = _plan(pr, "fp32")
    m = W.normal_model(pr, 9)
    v = W.normal_data(pr, 10)
    a = _products(torch_cuda, plan, m, v)
    b = _products(torch_cuda, plan, m, v)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_concurrent_calls_on_one_plan(torch_cuda):
    # one plan, four host threads, each with its own stream and workspace:
    # every result equals the sequential one bitwise
    import threading
    torch = torch_cuda
    from paper_1912_06976_amd import Plan, bttb_forward, bttb_transpose
    pr = W.magnetic_48x56()
    plan = _plan(pr, "fp32")
    m = torch.tensor(W.normal_model(pr, 91), dtype=torch.float32, device="cuda")
    v = torch.tensor(W.normal_data(pr, 92), dtype=torch.float32, device="cuda")
    ref_d, ref_t = plan.forward(m), plan.transpose(v)
    torch.cuda.synchronize()
    nws = plan.workspace_bytes(1)
    errors, outs = [], {}

    def work(k):
        try:
            s = torch.cuda.Stream()
            ws = torch.empty(nws, dtype=torch.uint8, device="cuda")
            d = torch.empty_like(ref_d)
            t = torch.empty_like(ref_t)
            for _ in range(5):
                bttb_forward(plan.handle, plan.spectra, m, d, 1, ws, s)
                bttb_transpose(plan.handle, plan.spectra, v, t, 1, ws, s)
            s.synchronize()
            outs[k] = (d, t)
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)
    th = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errors, errors
    for k in range(4):
        assert torch.equal(outs[k][0], ref_d) and torch.equal(outs[k][1], ref_t)


def test_plan_products_on_two_streams(torch_cuda):
    # one Plan driven from two streams at once: each stream has its own
    # workspace (allocated on it), so the products do not race and equal the
    # sequential results bitwise
    torch = torch_cuda
    pr = W.magnetic_48x56()
    plan = _plan(pr, "fp32")
    ms = [torch.tensor(W.normal_model(pr, 93 + k, nrhs=1 + k), dtype=torch.float32, device="cuda") for k in range(2)]
    vs = [torch.tensor(W.normal_data(pr, 95 + k, nrhs=1 + k), dtype=torch.float32, device="cuda") for k in range(2)]
    ref = [(plan.forward(m), plan.transpose(v)) for m, v in zip(ms, vs)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [[], []]
    for rep in range(4):
        for k, s in enumerate(streams):
            outs[k].append((plan.forward(ms[k], stream=s), plan.transpose(vs[k], stream=s)))
    torch.cuda.synchronize()
    assert len([key for key in plan._ws if key in (int(s.cuda_stream) for s in streams)]) == 2
    for k in range(2):
        for d, t in outs[k]:
            assert torch.equal(d, ref[k][0]) and torch.equal(t, ref[k][1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", [W.GRAVITY, W.MAGNETIC])
def test_forward_depth_split_many_layers(torch_cuda, orc, prec, kind):
    # few columns and 256 layers: the forward sums its layers in 64 ranges
    # (FP64 partial sums added by the finishing kernel), for one and for
    # several right-hand sides
    kw = dict(dx=20.0, dy=20.0, dz=5.0)
    if kind == W.MAGNETIC:
        kw.update(incl=50.0, decl=-30.0, field_nT=47000.0)
    pr = W.problem(kind, 6, 5, 256, 1, 2, 0, 1, **kw)
    _say("depth split", kind, prec)
    P = oracle_problem(pr)
    G = orc.dense_G_quad(P)
    Gp = orc.dense_G(P)
    tq, _ = orc.offset_table_quad(P)
    tol = TOL64 if prec == "fp64" else TOL32
    plan = _plan(pr, prec)
    from paper_1912_06976_amd import Plan
    plan_t = Plan(dict(pr, kind=W.TABLE), prec)
    plan_t.generate(table=torch_cuda.tensor(np.ascontiguousarray(tq), dtype=torch_cuda.float64, device="cuda"))
    for nrhs in (1, 3):
        m = W.normal_model(pr, 700 + nrhs, nrhs=nrhs)
        v = W.normal_data(pr, 800 + nrhs, nrhs=nrhs)
        # the exact entries as a table: the bar itself
        d, t = _products(torch_cuda, plan_t, m, v)
        assert rel_l2(d.reshape(nrhs, -1), m.reshape(nrhs, -1) @ G.T) <= tol
        assert rel_l2(t.reshape(nrhs, -1), v.reshape(nrhs, -1) @ G) <= tol
        # generated entries: the bar, or in FP64 10x the oracle's own
        # plain-FP64 error on the same product (the deepest prisms are 64
        # cells below the stations)
        d, t = _products(torch_cuda, plan, m, v)
        for q in range(nrhs):
            mq, vq = m[q].ravel(), v[q].ravel()
            bf = fp64_bar(Gp, G, mq) if prec == "fp64" else tol
            bt = fp64_bar(Gp, G, vq, transpose=True) if prec == "fp64" else tol
            assert rel_l2(d[q].ravel(), G @ mq) <= bf
            assert rel_l2(t[q].ravel(), G.T @ vq) <= bt


def test_empty_inputs_and_rhs_mismatch(torch_cuda):
    # no right-hand side: empty results, nothing launched; an output with a
    # different right-hand-side count is refused before any launch
    torch = torch_cuda
    pr = W.small_gravity()
    plan = _plan(pr, "fp32")
    m0 = torch.empty((0, plan.nz, plan.ny, plan.nx), device="cuda")
    r0 = torch.empty((0, plan.sy, plan.sx), device="cuda")
    assert tuple(plan.forward(m0).shape) == (0, plan.sy, plan.sx)
    assert tuple(plan.transpose(r0).shape) == (0, plan.nz, plan.ny, plan.nx)
    m2 = torch.zeros((2, plan.nz, plan.ny, plan.nx), device="cuda")
    r2 = torch.zeros((2, plan.sy, plan.sx), device="cuda")
    with pytest.raises(ValueError):
        plan.forward(m2, out=torch.empty((3, plan.sy, plan.sx), device="cuda"))
    with pytest.raises(ValueError):
        plan.transpose(r2, out=torch.empty((1, plan.nz, plan.ny, plan.nx), device="cuda"))
    torch.cuda.synchronize()
