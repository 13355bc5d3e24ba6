"""Seeded synthetic problem descriptions and inputs.

This module holds geometry parameters and random-number recipes only: it
contains none of the method's arithmetic, so both the CPU oracle (``oracle/``)
and the GPU library's tests and benchmark can draw their inputs from it.

The five workloads follow the shapes and value distributions of the paper's
experiments (Sec. 5: random model and data vectors on synthetic grids,
Table 1 sizes) scaled to the cases of interest:

* ``small_gravity``    16 x 16 x 8 prisms, 50 x 50 x 25 m, no padding;
* ``magnetic_48x56``   40 x 48 stations, 4 padding cells per side, 16 layers;
* ``gravity_1024``     1000 x 1000 stations, 12 padding cells per side,
                       1024 x 1024 x 128 prisms of 25 x 25 x 20 m;
* ``batch48``          48 seeded instances of mixed size and kind;
* ``magnetic_288``     256 x 256 stations, 16 padding cells, 48 layers
                       (and its 20 x 20, 2-cell-padding small check).

All arrays are generated in float64 on the host with numpy's PCG64.
"""
from __future__ import annotations

import math

import numpy as np

GRAVITY, MAGNETIC, TABLE, HESSIAN, PROBE = "gravity", "magnetic", "table", "hessian", "probe"


def problem(kind, sx, sy, nz, pxl=0, pxr=0, pyl=0, pyr=0, dx=1.0, dy=1.0, dz=1.0,
            z_edges=None, h=0.0, incl=90.0, decl=0.0, field_nT=50000.0, scale=0.0,
            nx_fft=0, ny_fft=0, hessian=None):
    """A plain dict describing one problem (the parameter set of Table 2;
    hessian: the six weights of a "hessian" kernel)."""
    return dict(kind=kind, sx=int(sx), sy=int(sy), nz=int(nz), pxl=int(pxl), pxr=int(pxr),
                pyl=int(pyl), pyr=int(pyr), dx=float(dx), dy=float(dy), dz=float(dz),
                z_edges=None if z_edges is None else np.asarray(z_edges, dtype=np.float64),
                h=float(h), incl=float(incl), decl=float(decl), field_nT=float(field_nT),
                scale=float(scale), nx_fft=int(nx_fft), ny_fft=int(ny_fft),
                hessian=None if hessian is None else tuple(float(v) for v in hessian))


def dims(pr):
    nx = pr["sx"] + pr["pxl"] + pr["pxr"]
    ny = pr["sy"] + pr["pyl"] + pr["pyr"]
    return nx, ny, pr["nz"]


def pad_rule(s, frac=0.05):
    """Padding cells per side: round(frac * s) with halves away from zero
    (the reading of the padding of Table 1 that reproduces its n column)."""
    return int(math.floor(frac * s + 0.5))


# --------------------------------------------------------------------------
# problem descriptions
# --------------------------------------------------------------------------

def small_gravity():
    return problem(GRAVITY, 16, 16, 8, dx=50.0, dy=50.0, dz=25.0)


def magnetic_48x56():
    return problem(MAGNETIC, 40, 48, 16, 4, 4, 4, 4, dx=100.0, dy=100.0, dz=50.0,
                   incl=60.0, decl=15.0, field_nT=47000.0)


def gravity_1024():
    return problem(GRAVITY, 1000, 1000, 128, 12, 12, 12, 12, dx=25.0, dy=25.0, dz=20.0)


def magnetic_288():
    return problem(MAGNETIC, 256, 256, 48, 16, 16, 16, 16, dx=100.0, dy=100.0, dz=50.0,
                   incl=60.0, decl=15.0, field_nT=47000.0)


def magnetic_24():
    return problem(MAGNETIC, 20, 20, 6, 2, 2, 2, 2, dx=100.0, dy=100.0, dz=50.0,
                   incl=60.0, decl=15.0, field_nT=47000.0)


def table1_problem(k, kind=GRAVITY, padded=False, **kw):
    """Problem k (1..12) of Table 1: (sx, sy, nz) = k * (25, 15, 2)."""
    sx, sy, nz = 25 * k, 15 * k, 2 * k
    px = pad_rule(sx) if padded else 0
    py = pad_rule(sy) if padded else 0
    return problem(kind, sx, sy, nz, px, px, py, py, **kw)


def batch48(seed=401):
    """48 instances: sx, sy ~ U{32..384}; each padding round(U[0, 0.10] s);
    nz ~ U{8..64}; dx = dy ~ U{25, 50, 100} m, dz = dx / 2; instances 0-23
    gravity, 24-47 magnetic with I ~ U[-90, 90], D ~ U[-180, 180], F = 47000."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(48):
        sx, sy = (int(v) for v in rng.integers(32, 385, size=2))
        fr = rng.uniform(0.0, 0.10, size=4)
        pxl, pxr = (int(math.floor(f * sx + 0.5)) for f in fr[:2])
        pyl, pyr = (int(math.floor(f * sy + 0.5)) for f in fr[2:])
        nz = int(rng.integers(8, 65))
        d = float(rng.choice([25.0, 50.0, 100.0]))
        if k < 24:
            out.append(problem(GRAVITY, sx, sy, nz, pxl, pxr, pyl, pyr, dx=d, dy=d, dz=d / 2))
        else:
            incl = float(rng.uniform(-90.0, 90.0))
            decl = float(rng.uniform(-180.0, 180.0))
            out.append(problem(MAGNETIC, sx, sy, nz, pxl, pxr, pyl, pyr, dx=d, dy=d, dz=d / 2,
                               incl=incl, decl=decl, field_nT=47000.0))
    return out


# --------------------------------------------------------------------------
# model and data vectors
# --------------------------------------------------------------------------

def uniform_model(pr, seed, lo=0.0, hi=1.0, nrhs=None):
    nx, ny, nz = dims(pr)
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx) if nrhs is None else (nrhs, nz, ny, nx)
    return rng.uniform(lo, hi, size=shape)


def normal_model(pr, seed, nrhs=None):
    nx, ny, nz = dims(pr)
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx) if nrhs is None else (nrhs, nz, ny, nx)
    return rng.standard_normal(shape)


def normal_data(pr, seed, nrhs=None):
    rng = np.random.default_rng(seed)
    shape = (pr["sy"], pr["sx"]) if nrhs is None else (nrhs, pr["sy"], pr["sx"])
    return rng.standard_normal(shape)


def box_model(pr, seed, nboxes=3, lo=0.01, hi=0.1, noise_std=0.0, ext_xy=(3, 12), ext_z=(2, 8)):
    """Zero background plus ``nboxes`` axis-aligned boxes of value U[lo, hi]
    (extents U{ext_xy} x U{ext_xy} x U{ext_z} cells, clipped to the grid,
    overlaps add) plus optional iid N(0, noise_std) noise."""
    nx, ny, nz = dims(pr)
    rng = np.random.default_rng(seed)
    m = np.zeros((nz, ny, nx))
    for _ in range(nboxes):
        ex = min(int(rng.integers(ext_xy[0], ext_xy[1] + 1)), nx)
        ey = min(int(rng.integers(ext_xy[0], ext_xy[1] + 1)), ny)
        ez = min(int(rng.integers(ext_z[0], ext_z[1] + 1)), nz)
        x0 = int(rng.integers(0, nx - ex + 1))
        y0 = int(rng.integers(0, ny - ey + 1))
        z0 = int(rng.integers(0, nz - ez + 1))
        m[z0:z0 + ez, y0:y0 + ey, x0:x0 + ex] += rng.uniform(lo, hi)
    if noise_std > 0:
        m += rng.normal(0.0, noise_std, size=m.shape)
    return m


def ellipsoid_model(pr, seed, count=20, lo=-0.5, hi=0.5, dtype=np.float64):
    """Sum of ``count`` axis-aligned ellipsoids with contrast U[lo, hi]:
    centres uniform in the volume, semi-axes U[2 %, 20 %] of the extent per
    axis, overlaps add."""
    nx, ny, nz = dims(pr)
    rng = np.random.default_rng(seed)
    m = np.zeros((nz, ny, nx), dtype=dtype)
    ext = np.array([nx, ny, nz], dtype=np.float64)
    for _ in range(count):
        c = rng.uniform(0.0, 1.0, size=3) * ext
        ax = rng.uniform(0.02, 0.20, size=3) * ext
        val = rng.uniform(lo, hi)
        lo_i = np.maximum(np.floor(c - ax).astype(int), 0)
        hi_i = np.minimum(np.ceil(c + ax).astype(int) + 1, [nx, ny, nz])
        xs = (np.arange(lo_i[0], hi_i[0]) + 0.5 - c[0]) / ax[0]
        ys = (np.arange(lo_i[1], hi_i[1]) + 0.5 - c[1]) / ax[1]
        zs = (np.arange(lo_i[2], hi_i[2]) + 0.5 - c[2]) / ax[2]
        inside = (zs[:, None, None] ** 2 + ys[None, :, None] ** 2 + xs[None, None, :] ** 2) <= 1.0
        m[lo_i[2]:hi_i[2], lo_i[1]:hi_i[1], lo_i[0]:hi_i[0]] += (val * inside).astype(dtype)
    return m


def sample_indices(seed, count, upper):
    """``count`` distinct seeded indices in [0, upper)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(upper, size=min(count, upper), replace=False))


def fullsize_samples(pr, nst, npr, seed=910):
    """Seeded sample of stations (i, j) and prisms (p, q, r) of a large
    problem: the corners of the station grid and of the volume, plus ``nst``
    stations and ``npr`` prisms drawn without replacement per axis."""
    nx, ny, nz = dims(pr)
    st = [(0, 0), (pr["sx"] - 1, pr["sy"] - 1)] + list(zip(sample_indices(seed, nst, pr["sx"]).tolist(),
                                                         sample_indices(seed + 1, nst, pr["sy"]).tolist()))
    pq = [(0, 0, 0), (nx - 1, ny - 1, nz - 1)] + list(zip(sample_indices(seed + 2, npr, nx).tolist(),
                                                        sample_indices(seed + 3, npr, ny).tolist(),
                                                        np.random.default_rng(seed + 4).integers(0, nz, npr).tolist()))
    return st, pq


def fullsize_case(name):
    """The large problems with their seeded inputs and sample sizes:
    (problem, m, r, stations, prisms)."""
    if name == "gravity_1024":
        pr = gravity_1024()
        m, r = ellipsoid_model(pr, 301), normal_data(pr, 302)
        st, pq = fullsize_samples(pr, 8, 32)
    elif name == "magnetic_288":
        pr = magnetic_288()
        m, r = box_model(pr, 501, nboxes=5), normal_data(pr, 502)
        st, pq = fullsize_samples(pr, 16, 48)
    else:
        raise KeyError(name)
    return pr, m, r, st, pq
