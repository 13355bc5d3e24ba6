"""Randomised pins of the oracle's prism formulas (hypothesis, derandomised,
CPU): the properties the fixed-case pins check, over drawn geometries and
field directions.  Each compares the oracle with an independent quantity or
with itself under an exact transformation of the geometry."""
import math

import numpy as np
import pytest
from hypothesis import assume, given, settings, strategies as st

from test_oracle_pins import field_dir, gauss_legendre_box, gz_integrand, tmi_integrand

EPS = np.finfo(float).eps
SETTINGS = settings(max_examples=40, derandomize=True, deadline=None, database=None)

coord = st.floats(-400.0, 400.0, allow_nan=False)
width = st.floats(5.0, 200.0, allow_nan=False)
depth = st.floats(0.5, 300.0, allow_nan=False)
frac = st.floats(0.1, 0.9, allow_nan=False)
incl = st.floats(-90.0, 90.0, allow_nan=False)
decl = st.floats(-180.0, 180.0, allow_nan=False)


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


@SETTINGS
@given(x1=coord, y1=coord, z1=depth, wx=width, wy=width, wz=width, fx=frac, fy=frac, fz=frac,
       kind=st.sampled_from([0, 1]), inc=incl, dec=decl)
def test_additivity_random(orc, x1, y1, z1, wx, wy, wz, fx, fy, fz, kind, inc, dec):
    # eight sub-prisms split at arbitrary interior planes sum to the prism
    # (corner terms telescope); values evaluated in __float128, rounded once
    xs = (x1, x1 + fx * wx, x1 + wx)
    ys = (y1, y1 + fy * wy, y1 + wy)
    assume(min(abs(v) for v in xs + ys) > 0.25)
    zs = (z1, z1 + fz * wz, z1 + wz)
    whole, _ = orc.prism_value(kind, (xs[0], xs[2], ys[0], ys[2], zs[0], zs[2]), inc, dec, 1.0, quad=True)
    parts = [orc.prism_value(kind, (xs[i], xs[i + 1], ys[j], ys[j + 1], zs[k], zs[k + 1]), inc, dec, 1.0,
                             quad=True)[0]
             for i in range(2) for j in range(2) for k in range(2)]
    tol = 16 * EPS * (sum(abs(p) for p in parts) + abs(whole))
    assert abs(sum(parts) - whole) <= tol


@SETTINGS
@given(x1=coord, y1=coord, wx=width, wy=width, wz=width, kind=st.sampled_from([0, 1]), inc=incl, dec=decl)
def test_quadrature_random(orc, x1, y1, wx, wy, wz, kind, inc, dec):
    # the closed forms against tensor Gauss-Legendre quadrature of the
    # integrands, for prisms whose top lies at least their largest width
    # below the station (smooth integrand over the prism)
    assume(min(abs(x1), abs(x1 + wx), abs(y1), abs(y1 + wy)) > 0.25)
    z1 = max(wx, wy, wz)
    box = (x1, x1 + wx, y1, y1 + wy, z1, z1 + wz)
    v, _ = orc.prism_value(kind, box, inc, dec, 1.0, quad=True)
    if kind == 0:
        q = gauss_legendre_box(gz_integrand, box, n=16, sub=2)
        assert abs(v - q) <= 1e-11 * abs(q)
    else:
        q = gauss_legendre_box(tmi_integrand(field_dir(inc, dec)), box, n=16, sub=2)
        scale = gauss_legendre_box(lambda X, Y, Z: 2.0 / (X * X + Y * Y + Z * Z) ** 1.5, box, 8, 1)
        assert abs(v - q) <= 1e-10 * scale


@SETTINGS
@given(x1=coord, y1=coord, z1=depth, wx=width, wy=width, wz=width, inc=incl, dec=decl)
def test_magnetic_symmetries_random(orc, x1, y1, z1, wx, wy, wz, inc, dec):
    # no horizontal edge through the station's vertical (on the product's
    # staggered grid an edge is never there; the closed form divides by it)
    assume(min(abs(x1), abs(x1 + wx), abs(y1), abs(y1 + wy)) > 0.25)
    box = np.array([x1, x1 + wx, y1, y1 + wy, z1, z1 + wz])
    mirror = np.array([-box[1], -box[0], -box[3], -box[2], box[4], box[5]])
    v, a = orc.prism_value(1, box, inc, dec, 1.0, quad=True)
    tol = 16 * EPS * a
    # D -> D + 180 (horizontal field reversed) equals the prism mirrored
    # through the station's vertical axis
    w, _ = orc.prism_value(1, mirror, inc, dec + 180.0, 1.0, quad=True)
    assert abs(v - w) <= tol
    # I -> -I together with D -> D + 180 reverses the whole field direction,
    # and the kernel is quadratic in it
    u, _ = orc.prism_value(1, box, -inc, dec + 180.0, 1.0, quad=True)
    assert abs(v - u) <= tol
    # rotating the prism by +90 deg about the vertical through the station
    # and the declination by +90 deg leaves the value unchanged
    rot = np.array([-box[3], -box[2], box[0], box[1], box[4], box[5]])
    r, _ = orc.prism_value(1, rot, inc, dec + 90.0, 1.0, quad=True)
    assert abs(v - r) <= tol


@SETTINGS
@given(x1=coord, y1=coord, z1=depth, wx=width, wy=width, wz=width)
def test_gravity_symmetries_random(orc, x1, y1, z1, wx, wy, wz):
    # g_z is even in x and in y and symmetric under exchanging x and y
    assume(min(abs(x1), abs(x1 + wx), abs(y1), abs(y1 + wy)) > 0.25)
    b = (x1, x1 + wx, y1, y1 + wy, z1, z1 + wz)
    v, a = orc.prism_value(0, b, scale=1.0, quad=True)
    tol = 16 * EPS * a
    for t in [(-b[1], -b[0], b[2], b[3]), (b[0], b[1], -b[3], -b[2]), (b[2], b[3], b[0], b[1])]:
        w, _ = orc.prism_value(0, (*t, b[4], b[5]), scale=1.0, quad=True)
        assert abs(v - w) <= tol
    assert v > 0.0


def test_field_direction_helper():
    # the test's own direction cosines: unit length, (L, M, N) convention
    f = field_dir(30.0, 45.0)
    assert abs(np.linalg.norm(f) - 1.0) < 1e-15
    assert abs(f[2] - math.sin(math.radians(30.0))) < 1e-15
