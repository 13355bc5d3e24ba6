"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests re-types the oracle's closed forms: each compares the
oracle with an independent quantity (numerical quadrature of the integrand,
far-field limits, exact potential-theory values, symmetries, the paper's
printed index examples and Table 1, a library FFT).
"""
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ----------------------------------------------------------------------------
# helpers (independent of the oracle)
# ----------------------------------------------------------------------------

def gauss_legendre_box(fun, box, n=24, sub=4):
    """Tensor Gauss-Legendre quadrature of fun(x, y, z) over box =
    (x1, x2, y1, y2, z1, z2), split into sub^3 cells."""
    x, w = np.polynomial.legendre.leggauss(n)
    edges = [np.linspace(box[2 * a], box[2 * a + 1], sub + 1) for a in range(3)]
    total = 0.0
    for i in range(sub):
        for j in range(sub):
            for k in range(sub):
                lo = (edges[0][i], edges[1][j], edges[2][k])
                hi = (edges[0][i + 1], edges[1][j + 1], edges[2][k + 1])
                pts = [0.5 * (hi[a] - lo[a]) * x + 0.5 * (hi[a] + lo[a]) for a in range(3)]
                ww = [0.5 * (hi[a] - lo[a]) * w for a in range(3)]
                X, Y, Z = np.meshgrid(*pts, indexing="ij")
                Wt = ww[0][:, None, None] * ww[1][None, :, None] * ww[2][None, None, :]
                total += float(np.sum(Wt * fun(X, Y, Z)))
    return total


def field_dir(incl, decl):
    I, D = math.radians(incl), math.radians(decl)
    return np.array([math.cos(I) * math.cos(D), math.cos(I) * math.sin(D), math.sin(I)])


def gz_integrand(X, Y, Z):
    # vertical attraction of a unit density element at (X, Y, Z) relative to
    # the station, z down: zeta / rho^3
    return Z / (X * X + Y * Y + Z * Z) ** 1.5


def tmi_integrand(f):
    # f^T (Hessian of 1/R) f = (3 (f.R)^2 - R^2) / R^5
    def fun(X, Y, Z):
        R2 = X * X + Y * Y + Z * Z
        fr = f[0] * X + f[1] * Y + f[2] * Z
        return (3.0 * fr * fr - R2) / R2 ** 2.5
    return fun


BOXES = [
    (-25.0, 25.0, -25.0, 25.0, 25.0, 50.0),      # directly below, one layer down
    (75.0, 125.0, -125.0, -75.0, 50.0, 75.0),    # offset diagonally, deeper
    (-25.0, 25.0, -25.0, 25.0, 5.0, 30.0),       # just below a raised station
    (-175.0, -125.0, 25.0, 75.0, 0.5, 25.5),     # shallow, to the side
    (425.0, 475.0, 925.0, 975.0, 100.0, 125.0),  # far
]


# ----------------------------------------------------------------------------
# closed forms against quadrature
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("box", BOXES)
def test_gravity_matches_quadrature(oracle_lib, box):
    v, _ = oracle_lib.prism_value(oracle_lib.GRAVITY, box, scale=1.0, quad=True)
    q = gauss_legendre_box(gz_integrand, box, n=24, sub=4)
    assert abs(v - q) <= 1e-12 * abs(q)


@pytest.mark.parametrize("incl,decl", [(60.0, 15.0), (0.0, 0.0), (0.0, 90.0), (90.0, 0.0),
                                       (-35.0, 140.0), (20.0, -110.0)])
@pytest.mark.parametrize("box", BOXES)
def test_magnetic_matches_quadrature(oracle_lib, box, incl, decl):
    # with F/(4 pi) = 1 the entry is f^T U f
    v, _ = oracle_lib.prism_value(oracle_lib.MAGNETIC, box, incl, decl, scale=1.0, quad=True)
    q = gauss_legendre_box(tmi_integrand(field_dir(incl, decl)), box, n=24, sub=4)
    scale = gauss_legendre_box(lambda X, Y, Z: 2.0 / (X * X + Y * Y + Z * Z) ** 1.5, box, 12, 2)
    assert abs(v - q) <= 1e-10 * scale


def test_double_and_quad_agree_near_field(oracle_lib):
    for box in BOXES:
        for kind in (oracle_lib.GRAVITY, oracle_lib.MAGNETIC):
            vd, a = oracle_lib.prism_value(kind, box, 60.0, 15.0, 1.0, quad=False)
            vq, _ = oracle_lib.prism_value(kind, box, 60.0, 15.0, 1.0, quad=True)
            assert abs(vd - vq) <= 32 * np.finfo(float).eps * a


# ----------------------------------------------------------------------------
# far-field limits
# ----------------------------------------------------------------------------

def test_gravity_point_mass_limit(oracle_lib):
    # a 50 x 50 x 25 m prism at growing distance behaves like a point mass
    # V zeta / R^3; the relative gap shrinks like (size / R)^2
    gaps = []
    for R in (400.0, 800.0, 1600.0, 3200.0):
        c = np.array([0.6 * R, 0.48 * R, 0.64 * R])  # |c| = R
        box = (c[0] - 25, c[0] + 25, c[1] - 25, c[1] + 25, c[2] - 12.5, c[2] + 12.5)
        v, _ = oracle_lib.prism_value(oracle_lib.GRAVITY, box, scale=1.0, quad=True)
        pm = 50 * 50 * 25 * c[2] / R ** 3
        gaps.append(abs(v - pm) / pm)
    for a, b in zip(gaps, gaps[1:]):
        assert 3.0 < a / b < 5.0          # second-order convergence
    assert gaps[-1] < 1e-4
    assert all(np.sign(gaps) >= 0)


def test_gravity_positive_below(oracle_lib):
    v, _ = oracle_lib.prism_value(oracle_lib.GRAVITY, (-25, 25, -25, 25, 0.0, 25.0), scale=1.0)
    assert v > 0
    v, _ = oracle_lib.prism_value(oracle_lib.GRAVITY, (300, 350, -25, 25, 0.0, 25.0), scale=1.0)
    assert v > 0


@pytest.mark.parametrize("incl,decl", [(60.0, 15.0), (-20.0, 100.0), (90.0, 0.0)])
def test_magnetic_dipole_limit(oracle_lib, incl, decl):
    f = field_dir(incl, decl)
    gaps = []
    for R in (800.0, 1600.0, 3200.0):
        c = np.array([0.36 * R, -0.48 * R, 0.8 * R])
        box = (c[0] - 50, c[0] + 50, c[1] - 50, c[1] + 50, c[2] - 25, c[2] + 25)
        v, _ = oracle_lib.prism_value(oracle_lib.MAGNETIC, box, incl, decl, scale=1.0, quad=True)
        Rh = c / R
        V = 100 * 100 * 50
        dip = V * (3.0 * (f @ Rh) ** 2 - 1.0) / R ** 3
        gaps.append(abs(v - dip) / (V / R ** 3))  # relative to the field scale
    # second-order convergence to the dipole field
    assert 3.5 < gaps[0] / gaps[1] < 4.5 and 3.5 < gaps[1] / gaps[2] < 4.5
    assert gaps[-1] < 1e-3


# ----------------------------------------------------------------------------
# exact values from potential theory
# ----------------------------------------------------------------------------

def test_bouguer_slab(oracle_lib):
    # one very wide thin prism right under the station: g_z -> 2 pi t
    # (per unit gamma and density); the edge effect is about t / half-width
    W2, t = 1.0e6, 25.0
    v, _ = oracle_lib.prism_value(oracle_lib.GRAVITY, (-W2, W2, -W2, W2, 0.0, t), scale=1.0,
                                  quad=True)
    assert abs(v - 2 * math.pi * t) / (2 * math.pi * t) < 2e-5
    assert v < 2 * math.pi * t


@pytest.mark.parametrize("incl", [60.0, 90.0, 0.0, -45.0])
def test_magnetic_self_term_air_side(oracle_lib, incl):
    # station at the centre of the top face of a square prism of thickness
    # a / 2: U_zz (air side) = 2 pi - (solid angle of the bottom face) = 4 pi / 3,
    # U_xx = U_yy = -2 pi / 3, off-diagonals vanish by symmetry; so the entry
    # is F (sin^2 I - cos^2 I / 2) / 3 for any declination.
    F = 47000.0
    for decl in (0.0, 15.0, 77.0):
        v, _ = oracle_lib.prism_value(oracle_lib.MAGNETIC, (-50, 50, -50, 50, 0.0, 50.0), incl, decl,
                                      scale=F / (4 * math.pi), quad=True)
        I = math.radians(incl)
        exact = F * (math.sin(I) ** 2 - 0.5 * math.cos(I) ** 2) / 3.0
        assert abs(v - exact) <= 1e-12 * F


def test_gravity_top_face_matches_quadrature_limit(oracle_lib):
    # station on the top face centre (zeta1 = 0): the closed form with the
    # zeta -> 0 limit must equal the limit of stations raised by eps
    top = oracle_lib.prism_value(oracle_lib.GRAVITY, (-25, 25, -25, 25, 0.0, 25.0), scale=1.0,
                                 quad=True)[0]
    vals = [oracle_lib.prism_value(oracle_lib.GRAVITY, (-25, 25, -25, 25, e, 25.0 + e), scale=1.0,
                                   quad=True)[0] for e in (1e-3, 1e-4, 1e-5)]
    assert abs(vals[-1] - top) < 1e-3 * abs(top)
    assert abs(vals[-1] - top) < abs(vals[0] - top)


# ----------------------------------------------------------------------------
# corner bookkeeping and symmetries
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [0, 1])
def test_additivity_of_subprisms(oracle_lib, kind):
    box = np.array([30.0, 130.0, -80.0, 20.0, 40.0, 90.0])
    whole, a = oracle_lib.prism_value(kind, box, 60.0, 15.0, 1.0, quad=True)
    mid = [(box[0] + box[1]) / 2, (box[2] + box[3]) / 2, (box[4] + box[5]) / 2]
    xs, ys, zs = (box[0], mid[0], box[1]), (box[2], mid[1], box[3]), (box[4], mid[2], box[5])
    parts = 0.0
    for i in range(2):
        for j in range(2):
            for k in range(2):
                parts += oracle_lib.prism_value(kind, (xs[i], xs[i + 1], ys[j], ys[j + 1], zs[k],
                                                       zs[k + 1]), 60.0, 15.0, 1.0, quad=True)[0]
    assert abs(parts - whole) <= 1e-14 * max(a, 1.0)
    # two layers of dz equal one of 2 dz
    upper = oracle_lib.prism_value(kind, (*box[:4], 40.0, 65.0), 60.0, 15.0, 1.0, quad=True)[0]
    lower = oracle_lib.prism_value(kind, (*box[:4], 65.0, 90.0), 60.0, 15.0, 1.0, quad=True)[0]
    assert abs(upper + lower - whole) <= 1e-14 * max(a, 1.0)


def _mag_problem(incl, decl, **kw):
    import oracle
    base = dict(kind=oracle.MAGNETIC, sx=6, sy=5, nz=2, pxl=2, pxr=1, pyl=1, pyr=2, dx=100.0,
                dy=100.0, dz=50.0, incl=incl, decl=decl, field_nT=47000.0)
    base.update(kw)
    return oracle.Problem(**base)


def test_magnetic_declination_flip_reverses_offsets(oracle_lib):
    # D -> D + 180 reverses the horizontal field component; the kernel then
    # equals the original kernel at the negated horizontal offset
    a = _mag_problem(60.0, 15.0)
    b = _mag_problem(60.0, 195.0)
    for (dx, dy, r) in [(1, 2, 0), (-3, 1, 1), (2, -2, 0), (0, 3, 1)]:
        # station (3, 2); prism offset (dx, dy) -> p = dx + pxl + i
        i, j = 3, 2
        va = oracle_lib.entry(a, i, j, dx + a.pxl + i, dy + a.pyl + j, r, quad=True)[0]
        vb = oracle_lib.entry(b, i, j, -dx + b.pxl + i, -dy + b.pyl + j, r, quad=True)[0]
        assert abs(va - vb) <= 1e-12 * abs(va)


def test_magnetic_vertical_field_is_even(oracle_lib):
    a = _mag_problem(90.0, 33.0)
    i, j = 3, 2
    for (dx, dy) in [(1, 2), (2, 1), (1, 0), (2, 2)]:
        vals = [oracle_lib.entry(a, i, j, sx * dx + a.pxl + i, sy * dy + a.pyl + j, 0, quad=True)[0]
                for sx in (1, -1) for sy in (1, -1)]
        assert max(vals) - min(vals) <= 1e-12 * abs(vals[0])


def test_magnetic_rotation_by_90_degrees(oracle_lib):
    # for square cells, turning the field by +90 deg declination turns the
    # kernel: h_{D+90}(dx, dy) = h_D(dy, -dx)
    a = _mag_problem(40.0, 10.0)
    b = _mag_problem(40.0, 100.0)
    i, j = 3, 2
    for (dx, dy) in [(1, 2), (-2, 1), (2, -1), (0, 1)]:
        vb = oracle_lib.entry(b, i, j, dx + b.pxl + i, dy + b.pyl + j, 1, quad=True)[0]
        va = oracle_lib.entry(a, i, j, dy + a.pxl + i, -dx + a.pyl + j, 1, quad=True)[0]
        assert abs(va - vb) <= 1e-12 * abs(va)


# ----------------------------------------------------------------------------
# dense matrix: structure, index map, table mapping
# ----------------------------------------------------------------------------

def _oracle_problem(pr):
    import oracle
    kind = {W.GRAVITY: oracle.GRAVITY, W.MAGNETIC: oracle.MAGNETIC, W.PROBE: oracle.PROBE}[pr["kind"]]
    return oracle.Problem(kind=kind, sx=pr["sx"], sy=pr["sy"], nz=pr["nz"], pxl=pr["pxl"],
                          pxr=pr["pxr"], pyl=pr["pyl"], pyr=pr["pyr"], dx=pr["dx"], dy=pr["dy"],
                          dz=pr["dz"], z_edges=pr["z_edges"], h=pr["h"], incl=pr["incl"],
                          decl=pr["decl"], field_nT=pr["field_nT"], scale=pr["scale"])


def test_gravity_unpadded_layers_are_symmetric_bttb(oracle_lib):
    P = _oracle_problem(W.small_gravity())
    G = oracle_lib.dense_G(P)
    _, A = oracle_lib.dense_G_quad(P, with_abs=True)
    L = P.nx * P.ny
    for r in range(P.nz):
        Gr = G[:, r * L:(r + 1) * L]
        Ar = A[:, r * L:(r + 1) * L]
        # symBTTB (Sec. 2.2.1): h(d) = h(-d); the two are evaluated from
        # mirrored corners, so equal up to the rounding of the corner sums
        assert np.all(np.abs(Gr - Gr.T) <= 32 * np.finfo(float).eps * Ar)
        B = Gr.reshape(P.sy, P.sx, P.ny, P.nx)
        # block Toeplitz: block (j, q) depends on q - j only; Toeplitz blocks
        for j in range(P.sy):
            for q in range(P.ny):
                blk = B[j, :, q, :]
                ref = B[0, :, q - j, :] if q >= j else B[j - q, :, 0, :]
                assert np.array_equal(blk, ref)
                for i in range(1, P.sx):
                    assert np.array_equal(blk[i, 1:], blk[i - 1, :-1])


def test_padded_magnetic_is_bttb_not_symmetric(oracle_lib):
    P = _oracle_problem(W.problem(W.MAGNETIC, 5, 4, 2, 2, 1, 1, 3, dx=100.0, dy=100.0, dz=50.0,
                                  incl=60.0, decl=15.0, field_nT=47000.0))
    G = oracle_lib.dense_G(P)
    L = P.nx * P.ny
    for r in range(P.nz):
        B = G[:, r * L:(r + 1) * L].reshape(P.sy, P.sx, P.ny, P.nx)
        # entries depend on (p - i, q - j) only: exact equality along diagonals
        for j in range(1, P.sy):
            for i in range(1, P.sx):
                assert np.array_equal(B[j, i, 1:, 1:], B[j - 1, i - 1, :-1, :-1])
    # not symmetric: h(d) != h(-d) for a generic field direction
    i, j = 2, 1
    a = G[j * P.sx + i, 0 * L + (1 + P.pyl + j) * P.nx + (2 + P.pxl + i)]
    b = G[j * P.sx + i, 0 * L + (-1 + P.pyl + j) * P.nx + (-2 + P.pxl + i)]
    assert abs(a - b) > 1e-3 * abs(a)


def _label_delta(label, symmetric):
    if label.startswith("gamma"):
        return [-(int(label[5:]) - 1)]
    k = int(label[1:]) - 1
    return [k, -k] if symmetric else [k]


def _read_examples():
    out, cur = {}, None
    for line in open(os.path.join(GOLDEN, "paper_index_examples.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "example":
            cur = tok[1]
            out[cur] = dict(kv.split("=") for kv in tok[2:])
            out[cur]["rows"] = []
        else:
            out[cur]["rows"].append((tok[0], tok[1:]))
    return out


@pytest.mark.parametrize("name", ["sym_padded", "nonsym_padded"])
def test_paper_padded_index_examples(oracle_lib, name):
    ex = _read_examples()[name]
    sx, pxl, pxr = int(ex["sx"]), int(ex["pxl"]), int(ex["pxr"])
    P = _oracle_problem(W.problem(W.PROBE, sx, 1, 1, pxl, pxr, 0, 0, dx=10.0, dy=10.0, dz=5.0))
    G = oracle_lib.dense_G(P)   # probe entries = x offset (y offset 0, layer 0)
    rows = [r for kind, r in ex["rows"] if kind == "row"]
    assert G.shape == (len(rows), len(rows[0]))
    sym = name.startswith("sym")
    for i, labels in enumerate(rows):
        for p, lab in enumerate(labels):
            assert int(G[i, p]) in _label_delta(lab, sym), (i, p, lab, G[i, p])


@pytest.mark.parametrize("pr", [W.small_gravity(),
                                W.problem(W.MAGNETIC, 7, 5, 3, 2, 1, 0, 3, dx=100.0, dy=50.0,
                                          dz=50.0, h=10.0, incl=60.0, decl=15.0,
                                          field_nT=47000.0),
                                W.problem(W.GRAVITY, 6, 9, 2, 0, 3, 2, 2, dx=25.0, dy=25.0,
                                          z_edges=[0.0, 15.0, 40.0])])
def test_dense_geometry_matches_quad_offset_table(oracle_lib, pr):
    # every double entry computed from the coordinates equals the quad value
    # at its offset to within the cancellation of its corner terms
    P = _oracle_problem(pr)
    G = oracle_lib.dense_G(P)
    Gq, A = oracle_lib.dense_G_quad(P, with_abs=True)
    assert np.all(np.abs(G - Gq) <= 32 * np.finfo(float).eps * A + 1e-300)


def test_probe_index_map_matches_geometry(oracle_lib):
    pr = W.problem(W.PROBE, 5, 4, 3, 2, 1, 1, 2, dx=25.0, dy=50.0, dz=10.0)
    P = _oracle_problem(pr)
    G = oracle_lib.dense_G(P)
    for k in range(P.m):
        i, j = k % P.sx, k // P.sx
        for l in range(P.n):
            r, rem = divmod(l, P.nx * P.ny)
            q, p = divmod(rem, P.nx)
            assert G[k, l] == (p - P.pxl - i) + 4096 * (q - P.pyl - j) + 2 ** 24 * r


def test_table1_sizes():
    for line in open(os.path.join(GOLDEN, "table1_sizes.txt")):
        if line.startswith("#"):
            continue
        k, sx, sy, nz, m, n0, n5 = map(int, line.split())
        p0, p5 = W.table1_problem(k), W.table1_problem(k, padded=True)
        assert (p0["sx"], p0["sy"], p0["nz"]) == (sx, sy, nz)
        assert sx * sy == m
        assert np.prod(W.dims(p0)) == n0
        got = int(np.prod(W.dims(p5)))
        sig = float("%.5g" % got)
        assert got == n5 or sig == n5, (k, got, n5)


# ----------------------------------------------------------------------------
# products: direct sums, FFT identity, adjoint
# ----------------------------------------------------------------------------

def test_station_and_prism_sums_match_dense(oracle_lib):
    pr = W.problem(W.MAGNETIC, 9, 7, 3, 2, 1, 1, 2, dx=50.0, dy=50.0, dz=25.0, incl=60.0,
                   decl=15.0, field_nT=47000.0, h=5.0)
    P = _oracle_problem(pr)
    G = oracle_lib.dense_G(P)
    m = W.normal_model(pr, 7)
    v = W.normal_data(pr, 8)
    st = [(0, 0), (8, 6), (3, 4), (5, 1)]
    ds = oracle_lib.station_sums(P, m, st)
    ref = G @ m.ravel()
    for (i, j), val in zip(st, ds):
        assert abs(val - ref[j * P.sx + i]) <= 1e-12 * np.abs(G[j * P.sx + i]) @ np.abs(m.ravel())
    pq = [(0, 0, 0), (11, 9, 2), (4, 3, 1)]
    ts = oracle_lib.prism_sums(P, v, pq)
    reft = G.T @ v.ravel()
    for (p, q, r), val in zip(pq, ts):
        l = r * P.nx * P.ny + q * P.nx + p
        assert abs(val - reft[l]) <= 1e-12 * np.abs(G[:, l]) @ np.abs(v.ravel())


def test_gravity_station_sum_matches_dense_gravity(oracle_lib):
    pr = W.problem(W.GRAVITY, 8, 6, 4, 1, 2, 2, 0, dx=25.0, dy=25.0, dz=20.0)
    P = _oracle_problem(pr)
    G = oracle_lib.dense_G(P)
    m = W.uniform_model(pr, 3)
    ref = G @ m.ravel()
    got = oracle_lib.station_sums(P, m, [(0, 0), (7, 5), (2, 3)])
    for (i, j), val in zip([(0, 0), (7, 5), (2, 3)], got):
        assert abs(val - ref[j * P.sx + i]) <= 1e-12 * abs(ref[j * P.sx + i])


def test_dense_product_equals_library_fft_convolution(oracle_lib):
    # the paper's claim that the transform path reproduces the dense product
    # to ~10 eps (Sec. 5) holds for the oracle's own entries: a 2-D circular
    # convolution by numpy.fft of the offset table equals G m and G^T r
    pr = W.magnetic_24()
    P = _oracle_problem(pr)
    G = oracle_lib.dense_G_quad(P)
    t, _ = oracle_lib.offset_table_quad(P)
    m = W.normal_model(pr, 11)
    v = W.normal_data(pr, 12)
    Nx, Ny = P.sx + P.nx - 1, P.sy + P.ny - 1
    # forward: d[j,i] = sum_{q,p} t[r][q-pyl-j + oy0][p-pxl-i + ox0] m[r,q,p]
    # = correlation; compute with FFTs of zero-embedded arrays
    d = np.zeros((P.sy, P.sx))
    tr = np.zeros((P.nz, P.ny, P.nx))
    for r in range(P.nz):
        K = np.zeros((Ny, Nx))
        K[:t.shape[1], :t.shape[2]] = t[r]
        M = np.zeros((Ny, Nx))
        M[:P.ny, :P.nx] = m[r]
        corr = np.fft.irfft2(np.conj(np.fft.rfft2(M)) * np.fft.rfft2(K), s=(Ny, Nx))
        # corr[a,b] = sum_{q,p} M[q,p] K[q+a, p+b]; offset index for (i, p) is
        # p - pxl - i + sx - 1 + pxl = p + (sx - 1 - i)
        d += corr[P.sy - 1 - np.arange(P.sy)][:, P.sx - 1 - np.arange(P.sx)]
        V = np.zeros((Ny, Nx))
        V[:P.sy, :P.sx] = v
        conv = np.fft.irfft2(np.fft.rfft2(V) * np.fft.rfft2(K), s=(Ny, Nx))
        tr[r] = conv[P.sy - 1:P.sy - 1 + P.ny, P.sx - 1:P.sx - 1 + P.nx]
    ref = G @ m.ravel()
    assert np.linalg.norm(d.ravel() - ref) <= 1e-13 * np.linalg.norm(ref)
    reft = G.T @ v.ravel()
    assert np.linalg.norm(tr.ravel() - reft) <= 1e-13 * np.linalg.norm(reft)
    # adjoint identity of the dense pair
    lhs = float(ref @ v.ravel())
    rhs = float(m.ravel() @ reft)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(ref) * np.linalg.norm(v)


def test_regularized_lsq_matches_svd_filter_factors_and_augmented_lstsq(oracle_lib):
    # the minimiser of ||G m - d||^2 + lam^2 ||m||^2 has the closed form
    # sum_i s_i / (s_i^2 + lam^2) (u_i^T d) v_i (Tikhonov filter factors) and
    # is the least-squares solution of the stacked system [G; lam I] m = [d; 0]
    import oracle
    import scipy.linalg
    P = oracle.problem_from_dict(W.small_gravity())
    G = oracle.dense_G(P)
    rng = np.random.default_rng(5)
    d = G @ rng.uniform(0, 1, G.shape[1]) + 0.01 * rng.standard_normal(G.shape[0])
    U, sv, Vt = np.linalg.svd(G, full_matrices=False)
    for lam in (0.3 * sv[0], 0.05 * sv[0], 1e-3 * sv[0]):
        m = oracle.regularized_lsq(G, d, lam)
        m_svd = Vt.T @ (sv / (sv ** 2 + lam ** 2) * (U.T @ d))
        A = np.vstack([G, lam * np.eye(G.shape[1])])
        m_ls = scipy.linalg.lstsq(A, np.concatenate([d, np.zeros(G.shape[1])]))[0]
        for other in (m_svd, m_ls):
            assert np.linalg.norm(m - other) <= 1e-9 * np.linalg.norm(other)
    # a large lam gives m -> G^T d / lam^2
    lam = 1e4 * sv[0]
    m = oracle.regularized_lsq(G, d, lam)
    ref = G.T @ d / lam ** 2
    assert np.linalg.norm(m - ref) <= 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("pr", [W.small_gravity(), W.magnetic_48x56(),
                                W.problem(W.MAGNETIC, 9, 6, 3, 1, 2, 2, 1, dx=50.0, dy=100.0, dz=30.0,
                                          h=7.0, incl=-30.0, decl=140.0, field_nT=52000.0)])
def test_dense_from_table_reproduces_geometry_entries(oracle_lib, pr):
    # the offsets table of the exact entries, indexed by cell offset, gives
    # back the matrix assembled from the station and prism coordinates
    import oracle
    P = oracle.problem_from_dict(pr)
    t, _ = oracle.offset_table_quad(P)
    assert np.array_equal(oracle.dense_from_table(pr, t), oracle.dense_G_quad(P))


# ----------------------------------------------------------------------------
# station height
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("h", [7.5, 40.0])
def test_station_height_entries_match_quadrature(oracle_lib, h):
    # A raised station at c = -h sees the prism's depth range [z_r, z_{r+1}]
    # at vertical distances [z_r + h, z_{r+1} + h].  The box is built here
    # from the station and prism coordinates (Table 3) and the integrand is
    # integrated by quadrature; the oracle's entries (through the problem's
    # station height, in double and in quad, and its dense matrix) must agree.
    # A slip in the sign or placement of h moves the box and fails this.
    import oracle
    for kind, kw in ((oracle.GRAVITY, {}), (oracle.MAGNETIC, dict(incl=50.0, decl=-25.0))):
        P = oracle.Problem(kind=kind, sx=5, sy=4, nz=3, pxl=1, pxr=2, pyl=2, pyr=0, dx=40.0, dy=30.0,
                           z_edges=np.array([0.0, 10.0, 35.0, 50.0]), h=h, scale=1.0, **kw)
        G = oracle_lib.dense_G(P)
        z = P.zedges()
        for (i, j, p, q, r) in [(0, 0, 1, 2, 0), (3, 2, 0, 5, 1), (4, 3, 7, 1, 2), (2, 1, 3, 3, 0)]:
            a, b = (i + 0.5) * P.dx, (j + 0.5) * P.dy
            box = ((p - P.pxl) * P.dx - a, (p - P.pxl + 1) * P.dx - a,
                   (q - P.pyl) * P.dy - b, (q - P.pyl + 1) * P.dy - b,
                   z[r] - (-h), z[r + 1] - (-h))
            fun = gz_integrand if kind == oracle.GRAVITY else tmi_integrand(field_dir(P.incl, P.decl))
            ref = gauss_legendre_box(fun, box, n=24, sub=4)
            vq, _ = oracle_lib.entry(P, i, j, p, q, r, quad=True)
            vd, _ = oracle_lib.entry(P, i, j, p, q, r, quad=False)
            gd = G[j * P.sx + i, r * P.nx * P.ny + q * P.nx + p]
            for v in (vq, vd, gd):
                assert abs(v - ref) <= 1e-10 * abs(ref), (kind, i, j, p, q, r, v, ref)
        # and a station height of 0 gives a different entry (h is used)
        P0 = oracle.Problem(**{**P.__dict__, "h": 0.0, "_keep": []})
        assert abs(oracle_lib.entry(P0, 0, 0, 1, 2, 0)[0] - oracle_lib.entry(P, 0, 0, 1, 2, 0)[0]) > 1e-3 * abs(
            oracle_lib.entry(P, 0, 0, 1, 2, 0)[0])


def test_quad_direct_sums_match_dense_quad_matrix(oracle_lib):
    # the __float128 row and column sums against the dense matrix of quad
    # entries (summed exactly here with math.fsum)
    import math as _m
    import oracle
    for pr in (W.problem(W.MAGNETIC, 9, 7, 3, 2, 1, 1, 2, dx=50.0, dy=50.0, dz=25.0, incl=60.0, decl=15.0,
                         field_nT=47000.0, h=5.0),
               W.problem(W.GRAVITY, 8, 6, 4, 1, 2, 2, 0, dx=25.0, dy=25.0, dz=20.0, h=2.0)):
        P = oracle.problem_from_dict(pr)
        Gq = oracle_lib.dense_G_quad(P)
        m = W.normal_model(pr, 17).ravel()
        v = W.normal_data(pr, 18).ravel()
        st = [(0, 0), (P.sx - 1, P.sy - 1), (3, 2)]
        pq = [(0, 0, 0), (P.nx - 1, P.ny - 1, P.nz - 1), (4, 3, 1)]
        ds = oracle_lib.station_sums(P, m, st, quad=True)
        ts = oracle_lib.prism_sums(P, v, pq, quad=True)
        for (i, j), val in zip(st, ds):
            row = Gq[j * P.sx + i]
            ref = _m.fsum(row * m)
            assert abs(val - ref) <= 1e-14 * (np.abs(row) @ np.abs(m))
        for (p, q, r), val in zip(pq, ts):
            col = Gq[:, r * P.nx * P.ny + q * P.nx + p]
            ref = _m.fsum(col * v)
            assert abs(val - ref) <= 1e-14 * (np.abs(col) @ np.abs(v))
