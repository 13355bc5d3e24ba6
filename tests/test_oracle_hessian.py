"""Pins of the oracle's "hessian" kernel, sum_ab w_ab U_ab with U_ab the
second derivatives of a prism's Newtonian potential with respect to the
station (the user-chosen kernels of Sec. 1 (vi): gravity gradients, the
anomaly of a remanent magnetisation, field components), against quantities
that do not come from its closed forms: quadrature of each component's
integrand, Laplace's equation, the far-field dipole, the exact air-side value
on a face, the induced-magnetisation kernel of Sec. 4.2 as the special case
w = f f^T, and the parities of the components."""
import math

import numpy as np
import pytest

from test_oracle_pins import BOXES, field_dir, gauss_legendre_box

COMPONENTS = ["xx", "yy", "zz", "xy", "xz", "yz"]


def unit_weights(comp):
    return tuple(1.0 if c == comp else 0.0 for c in COMPONENTS)


def hessian_integrand(a, b):
    # d_a d_b (1 / R) = (3 R_a R_b - R^2 delta_ab) / R^5 (the station relative
    # to the element enters squared: either sign of R gives the same)
    ia, ib = "xyz".index(a), "xyz".index(b)

    def fun(X, Y, Z):
        C = (X, Y, Z)
        R2 = X * X + Y * Y + Z * Z
        return (3.0 * C[ia] * C[ib] - (R2 if ia == ib else 0.0)) / R2 ** 2.5
    return fun


def sym_weights(f, m):
    """w_aa = f_a m_a, w_ab = f_a m_b + f_b m_a (independent of the package)."""
    return (f[0] * m[0], f[1] * m[1], f[2] * m[2], f[0] * m[1] + f[1] * m[0], f[0] * m[2] + f[2] * m[0],
            f[1] * m[2] + f[2] * m[1])


def _scale(box):
    return gauss_legendre_box(lambda X, Y, Z: 2.0 / (X * X + Y * Y + Z * Z) ** 1.5, box, 12, 2)


@pytest.mark.parametrize("comp", COMPONENTS)
@pytest.mark.parametrize("box", BOXES)
def test_component_matches_quadrature(oracle_lib, box, comp):
    v, _ = oracle_lib.prism_value(oracle_lib.HESSIAN, box, scale=1.0, quad=True, w=unit_weights(comp))
    q = gauss_legendre_box(hessian_integrand(comp[0], comp[1]), box, n=24, sub=4)
    assert abs(v - q) <= 1e-10 * _scale(box), (comp, v, q)


@pytest.mark.parametrize("box", BOXES)
def test_laplace_trace_vanishes_outside(oracle_lib, box):
    # U_xx + U_yy + U_zz = 0 outside the prism (every box lies below the station)
    v, a = oracle_lib.prism_value(oracle_lib.HESSIAN, box, scale=1.0, quad=True, w=(1, 1, 1, 0, 0, 0))
    assert abs(v) <= 1e-25 * max(a, 1.0) + 1e-14 * _scale(box)


@pytest.mark.parametrize("incl,decl", [(60.0, 15.0), (-35.0, 140.0), (90.0, 0.0), (0.0, 90.0)])
@pytest.mark.parametrize("box", BOXES)
def test_induced_case_equals_the_magnetic_kernel(oracle_lib, box, incl, decl):
    # w = f f^T gives f^T U f, the induced total-field kernel of Sec. 4.2 (which
    # the oracle evaluates with U_zz eliminated by Laplace's equation)
    f = field_dir(incl, decl)
    v, _ = oracle_lib.prism_value(oracle_lib.HESSIAN, box, scale=1.0, quad=True, w=sym_weights(f, f))
    t, _ = oracle_lib.prism_value(oracle_lib.MAGNETIC, box, incl, decl, scale=1.0, quad=True)
    assert abs(v - t) <= 1e-25 + 1e-14 * _scale(box)


@pytest.mark.parametrize("fd,md", [((60.0, 15.0), (-30.0, 100.0)), ((90.0, 0.0), (0.0, 0.0)),
                                   ((20.0, -110.0), (75.0, 40.0))])
def test_remanent_dipole_limit(oracle_lib, fd, md):
    # far away the prism acts as a dipole of moment V m: f^T U m tends to
    # V (3 (f.R^)(m.R^) - f.m) / R^3 with a relative gap of order (size / R)^2
    f, m = field_dir(*fd), field_dir(*md)
    w = sym_weights(f, m)
    gaps = []
    for R in (800.0, 1600.0, 3200.0):
        c = np.array([0.36 * R, -0.48 * R, 0.8 * R])
        box = (c[0] - 50, c[0] + 50, c[1] - 50, c[1] + 50, c[2] - 25, c[2] + 25)
        v, _ = oracle_lib.prism_value(oracle_lib.HESSIAN, box, scale=1.0, quad=True, w=w)
        u = c / R
        dip = 100 * 100 * 50 * (3 * (f @ u) * (m @ u) - f @ m) / R ** 3
        gaps.append(abs(v - dip) / abs(dip))
    for a, b in zip(gaps, gaps[1:]):
        assert 3.0 < a / b < 5.0
    assert gaps[-1] < 1e-3


def test_air_side_values_on_the_top_face(oracle_lib):
    # station at the centre of the top face of a square cell of thickness half
    # its width (h = 0): the bottom face subtends 4 asin(1/2) = 2 pi / 3, so
    # U_zz = 2 pi - 2 pi / 3 = 4 pi / 3 from the air side, and by symmetry and
    # Laplace's equation U_xx = U_yy = -2 pi / 3; the off-diagonal ones vanish
    box = (-50.0, 50.0, -50.0, 50.0, 0.0, 50.0)
    want = {"zz": 4 * math.pi / 3, "xx": -2 * math.pi / 3, "yy": -2 * math.pi / 3, "xy": 0.0, "xz": 0.0, "yz": 0.0}
    for comp, val in want.items():
        v, _ = oracle_lib.prism_value(oracle_lib.HESSIAN, box, scale=1.0, quad=True, w=unit_weights(comp))
        assert abs(v - val) <= 1e-15, (comp, v, val)


@pytest.mark.parametrize("box", BOXES)
def test_component_parities(oracle_lib, box):
    # mirroring the prism in x (chi -> -chi) keeps U_xx, U_yy, U_zz, U_yz and
    # flips U_xy, U_xz; mirroring in y flips U_xy and U_yz
    mx = (-box[1], -box[0], box[2], box[3], box[4], box[5])
    my = (box[0], box[1], -box[3], -box[2], box[4], box[5])
    for comp in COMPONENTS:
        w = unit_weights(comp)
        v, _ = oracle_lib.prism_value(oracle_lib.HESSIAN, box, scale=1.0, quad=True, w=w)
        vx, _ = oracle_lib.prism_value(oracle_lib.HESSIAN, mx, scale=1.0, quad=True, w=w)
        vy, _ = oracle_lib.prism_value(oracle_lib.HESSIAN, my, scale=1.0, quad=True, w=w)
        sx = -1.0 if "x" in comp and comp != "xx" else 1.0
        sy = -1.0 if "y" in comp and comp != "yy" else 1.0
        tol = 1e-14 * _scale(box)
        assert abs(vx - sx * v) <= tol and abs(vy - sy * v) <= tol, comp


def test_double_and_quad_agree(oracle_lib):
    w = sym_weights(field_dir(60.0, 15.0), field_dir(-30.0, 100.0))
    for box in BOXES:
        vd, a = oracle_lib.prism_value(oracle_lib.HESSIAN, box, scale=1.0, quad=False, w=w)
        vq, _ = oracle_lib.prism_value(oracle_lib.HESSIAN, box, scale=1.0, quad=True, w=w)
        assert abs(vd - vq) <= 32 * np.finfo(float).eps * a


def test_package_weight_helpers_match():
    # the package's descriptor helpers give the same weights as this file's
    # independent construction
    from paper_1912_06976_amd import hessian_weights_component, hessian_weights_tmi
    assert np.allclose(hessian_weights_tmi(60.0, 15.0, -30.0, 100.0),
                       sym_weights(field_dir(60.0, 15.0), field_dir(-30.0, 100.0)), rtol=0, atol=1e-15)
    for comp in COMPONENTS:
        assert hessian_weights_component(comp[0], comp[1]) == unit_weights(comp)
        assert hessian_weights_component(comp[1], comp[0]) == unit_weights(comp)
