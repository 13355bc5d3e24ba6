"""CPU oracle for the gravity / magnetic BTTB products.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1912_06976_amd``) and never imports it.

What it computes is the plain definition of the products (Sec. 2,
eq. continuousforwardmodel / eq. Gslice of Hogue, Renaut & Vatankhah):

* ``dense_G``      -- every entry G[k, l] of the m x n sensitivity matrix from
                      the station and prism coordinates (C, double);
* ``dense_G_quad`` -- the same entries evaluated in __float128 and rounded
                      once (C), used as the exact reference for FP64 parity;
* ``forward`` / ``transpose`` -- d = G m and G^T r by a library matmul on the
                      dense matrix (Sec. 5: the direct products the paper
                      compares against);
* ``station_sums`` / ``prism_sums`` -- single rows / columns of G m and G^T r
                      for volumes too large for a dense G, in double or (quad)
                      entirely in __float128;
* ``regularized_lsq`` -- the minimiser of ||G m - d||^2 + lam^2 ||m||^2 from
                      the dense normal equations (checks the inversion driver);
* ``dense_from_table`` -- dense G of a kernel given by its entries per layer
                      and cell offset (checks user-supplied kernels).

The magnetic kernel is the total-field anomaly of induced magnetisation
(Sec. 4.2); the gravity kernel is g_z (Sec. 4.1); the "hessian" kernel is a
weighted sum of the second derivatives U_ab of the prism's potential with
respect to the station, each from its own closed form (user-chosen kernels,
Sec. 1 (vi)).  Conventions (0-based):
station (i, j) at ((i+1/2) dx, (j+1/2) dy, -h); prism (p, q, r) spans
[(p-pxl) dx, (p-pxl+1) dx] x [(q-pyl) dy, (q-pyl+1) dy] x [z_r, z_{r+1}] with z
down (Table 3); k = j sx + i and l = r nx ny + q nx + p (eq. htilde).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "prism_oracle.c")
_INC = os.path.join(_HERE, "prism_terms.inc")
_LIB = os.path.join(_HERE, "_prism_oracle.so")

GRAVITY, MAGNETIC, PROBE, HESSIAN = 0, 1, 2, 3

#: gravitational constant (CODATA 2018) converted so that density in g/cm^3
#: and lengths in m give g_z in mGal: 6.6743e-11 * 1e3 (g/cm^3 -> kg/m^3) *
#: 1e5 (m/s^2 -> mGal).
GAMMA_MGAL = 6.6743e-11 * 1e3 * 1e5


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, OpenMP, libquadmath) into ``_prism_oracle.so``."""
    if not force and os.path.exists(_LIB):
        if os.path.getmtime(_LIB) >= max(os.path.getmtime(_SRC), os.path.getmtime(_INC)):
            return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
           "-shared", "-fPIC", "-o", tmp, _SRC, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("sx", ctypes.c_int32), ("sy", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("pxl", ctypes.c_int32), ("pxr", ctypes.c_int32),
        ("pyl", ctypes.c_int32), ("pyr", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("h", ctypes.c_double),
        ("zedge", ctypes.POINTER(ctypes.c_double)),
        ("incl", ctypes.c_double), ("decl", ctypes.c_double), ("scale", ctypes.c_double),
        ("w", ctypes.c_double * 6),
    ]


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        # ORACLE_LIB: an instrumented build of the same source (sanitizer test)
        path = os.environ.get("ORACLE_LIB") or build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        pp = ctypes.POINTER(_Problem)
        L.orc_prism_value.restype = ctypes.c_double
        L.orc_prism_value.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, dp,
                                      ctypes.c_double, ctypes.c_int, dp]
        L.orc_dense_G.restype = ctypes.c_int
        L.orc_dense_G.argtypes = [pp, dp]
        L.orc_entry.restype = ctypes.c_double
        L.orc_entry.argtypes = [pp] + [ctypes.c_int] * 6 + [dp]
        L.orc_offset_table_quad.restype = ctypes.c_int
        L.orc_offset_table_quad.argtypes = [pp, dp, dp]
        L.orc_station_sums.restype = ctypes.c_int
        L.orc_station_sums.argtypes = [pp, dp, ctypes.c_int, ip, dp]
        L.orc_prism_sums.restype = ctypes.c_int
        L.orc_prism_sums.argtypes = [pp, dp, ctypes.c_int, ip, dp]
        L.orc_station_sums_quad.restype = ctypes.c_int
        L.orc_station_sums_quad.argtypes = [pp, dp, ctypes.c_int, ip, dp]
        L.orc_prism_sums_quad.restype = ctypes.c_int
        L.orc_prism_sums_quad.argtypes = [pp, dp, ctypes.c_int, ip, dp]
        _lib_handle = L
    return _lib_handle


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class Problem:
    """Geometry and physics of one problem (the parameter set of Table 2)."""
    kind: int
    sx: int
    sy: int
    nz: int
    pxl: int = 0
    pxr: int = 0
    pyl: int = 0
    pyr: int = 0
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    z_edges: np.ndarray | None = None
    h: float = 0.0
    incl: float = 90.0
    decl: float = 0.0
    field_nT: float = 50000.0
    scale: float = 0.0
    w: tuple = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)   # HESSIAN: w_xx, w_yy, w_zz, w_xy, w_xz, w_yz
    _keep: list = field(default_factory=list, repr=False)

    @property
    def nx(self) -> int:
        return self.sx + self.pxl + self.pxr

    @property
    def ny(self) -> int:
        return self.sy + self.pyl + self.pyr

    @property
    def m(self) -> int:
        return self.sx * self.sy

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def zedges(self) -> np.ndarray:
        if self.z_edges is not None:
            z = np.ascontiguousarray(self.z_edges, dtype=np.float64)
            assert z.shape == (self.nz + 1,)
            return z
        return np.arange(self.nz + 1, dtype=np.float64) * self.dz

    def effective_scale(self) -> float:
        if self.scale != 0.0:
            return self.scale
        if self.kind == GRAVITY:
            return GAMMA_MGAL
        if self.kind == MAGNETIC:
            return self.field_nT / (4.0 * math.pi)  # H~ = F / (4 pi), Table 2
        return 1.0

    def c_struct(self) -> _Problem:
        z = self.zedges()
        self._keep[:] = [z]
        return _Problem(self.kind, self.sx, self.sy, self.nz, self.pxl, self.pxr, self.pyl,
                        self.pyr, self.dx, self.dy, self.h, _dptr(z), self.incl, self.decl,
                        self.effective_scale(), (ctypes.c_double * 6)(*[float(v) for v in self.w]))


def problem_from_dict(pr: dict) -> Problem:
    """Problem from a plain description dict (keys as in workloads.problem)."""
    kind = {"gravity": GRAVITY, "magnetic": MAGNETIC, "probe": PROBE, "hessian": HESSIAN}[pr["kind"]]
    w = tuple(pr.get("hessian") or (0.0,) * 6)
    return Problem(kind=kind, sx=pr["sx"], sy=pr["sy"], nz=pr["nz"], pxl=pr["pxl"], pxr=pr["pxr"],
                   pyl=pr["pyl"], pyr=pr["pyr"], dx=pr["dx"], dy=pr["dy"], dz=pr["dz"],
                   z_edges=pr["z_edges"], h=pr["h"], incl=pr["incl"], decl=pr["decl"],
                   field_nT=pr["field_nT"], scale=pr["scale"], w=w)


def prism_value(kind: int, b, incl: float = 90.0, decl: float = 0.0, scale: float = 1.0,
                quad: bool = False, w=None):
    """scale * signed 8-corner sum for one prism b = (chi1, chi2, ups1, ups2, zeta1, zeta2)
    relative to the station (kind HESSIAN: with the component weights w).
    Returns (value, sum of |corner terms| * |scale|)."""
    bb = np.ascontiguousarray(b, dtype=np.float64)
    ww = np.ascontiguousarray(w if w is not None else np.zeros(6), dtype=np.float64)
    assert ww.shape == (6,)
    a = ctypes.c_double(0.0)
    v = _lib().orc_prism_value(kind, _dptr(bb), incl, decl, _dptr(ww), scale, int(quad), ctypes.byref(a))
    return v, a.value


def entry(P: Problem, i: int, j: int, p: int, q: int, r: int, quad: bool = False):
    """G[(i,j),(p,q,r)] and its sum of |corner terms|."""
    ps = P.c_struct()
    a = ctypes.c_double(0.0)
    v = _lib().orc_entry(ctypes.byref(ps), i, j, p, q, r, int(quad), ctypes.byref(a))
    return v, a.value


def dense_G(P: Problem) -> np.ndarray:
    """Dense m x n G, every entry from the geometry in double."""
    G = np.empty((P.m, P.n), dtype=np.float64)
    ps = P.c_struct()
    _lib().orc_dense_G(ctypes.byref(ps), _dptr(G))
    return G


def offset_table_quad(P: Problem):
    """Entries in __float128 (rounded once) for every offset (p-pxl-i, q-pyl-j, r);
    returns (table[nz][wy][wx], abs_table) with wx = sx + nx - 1, wy = sy + ny - 1."""
    wx, wy = P.sx + P.nx - 1, P.sy + P.ny - 1
    t = np.empty((P.nz, wy, wx), dtype=np.float64)
    a = np.empty_like(t)
    ps = P.c_struct()
    _lib().orc_offset_table_quad(ctypes.byref(ps), _dptr(t), _dptr(a))
    return t, a


def offsets(P: Problem):
    """Integer offset maps: for station k and prism column l (within a layer),
    ox[k, l] = p - pxl - i + (sx - 1 + pxl), oy likewise."""
    i = np.arange(P.sx)[None, :, None, None]
    j = np.arange(P.sy)[:, None, None, None]
    p = np.arange(P.nx)[None, None, None, :]
    q = np.arange(P.ny)[None, None, :, None]
    ox = (p - P.pxl - i) + (P.sx - 1 + P.pxl)
    oy = (q - P.pyl - j) + (P.sy - 1 + P.pyl)
    ox = np.broadcast_to(ox, (P.sy, P.sx, P.ny, P.nx)).reshape(P.m, P.nx * P.ny)
    oy = np.broadcast_to(oy, (P.sy, P.sx, P.ny, P.nx)).reshape(P.m, P.nx * P.ny)
    return ox, oy


def dense_G_quad(P: Problem, with_abs: bool = False):
    """Dense G whose entries are evaluated in __float128 and rounded once."""
    t, a = offset_table_quad(P)
    ox, oy = offsets(P)
    G = np.empty((P.m, P.n), dtype=np.float64)
    A = np.empty_like(G) if with_abs else None
    L = P.nx * P.ny
    for r in range(P.nz):
        G[:, r * L:(r + 1) * L] = t[r][oy, ox]
        if with_abs:
            A[:, r * L:(r + 1) * L] = a[r][oy, ox]
    return (G, A) if with_abs else G


def forward(G: np.ndarray, m: np.ndarray) -> np.ndarray:
    """d = G m for m of shape [..., nz, ny, nx]; returns [..., sy, sx] given P shapes by caller."""
    return m.reshape(-1, G.shape[1]) @ G.T


def transpose(G: np.ndarray, v: np.ndarray) -> np.ndarray:
    """G^T v for v of shape [..., sy, sx] (flattened per RHS)."""
    return v.reshape(-1, G.shape[0]) @ G


def station_sums(P: Problem, m: np.ndarray, stations, quad: bool = False) -> np.ndarray:
    """(G m)[k] at the given (i, j) stations without forming G; m is [nz][ny][nx].
    quad: corner terms and sums in __float128, rounded once (the exact reference)."""
    mm = np.ascontiguousarray(m, dtype=np.float64).reshape(P.nz, P.ny, P.nx)
    ij = np.ascontiguousarray(np.asarray(stations, dtype=np.int32).reshape(-1, 2))
    out = np.empty(ij.shape[0], dtype=np.float64)
    ps = P.c_struct()
    fn = _lib().orc_station_sums_quad if quad else _lib().orc_station_sums
    rc = fn(ctypes.byref(ps), _dptr(mm), ij.shape[0], _iptr(ij), _dptr(out))
    if rc != 0:
        raise RuntimeError("orc_station_sums failed (%d)" % rc)
    return out


def prism_sums(P: Problem, v: np.ndarray, prisms, quad: bool = False) -> np.ndarray:
    """(G^T v)[l] at the given (p, q, r) prisms without forming G; v is [sy][sx].
    quad: entries and sums in __float128, rounded once (the exact reference)."""
    vv = np.ascontiguousarray(v, dtype=np.float64).reshape(P.sy, P.sx)
    pqr = np.ascontiguousarray(np.asarray(prisms, dtype=np.int32).reshape(-1, 3))
    out = np.empty(pqr.shape[0], dtype=np.float64)
    ps = P.c_struct()
    fn = _lib().orc_prism_sums_quad if quad else _lib().orc_prism_sums
    rc = fn(ctypes.byref(ps), _dptr(vv), pqr.shape[0], _iptr(pqr), _dptr(out))
    if rc != 0:
        raise RuntimeError("orc_prism_sums failed (%d)" % rc)
    return out


def regularized_lsq(G: np.ndarray, d: np.ndarray, lam: float) -> np.ndarray:
    """The minimiser of ||G m - d||^2 + lam^2 ||m||^2 (the regularised inverse
    problem the transpose product serves, Sec. 1 and Sec. 7): the solution of
    the normal equations (G^T G + lam^2 I) m = G^T d by a dense FP64 solve."""
    G = np.asarray(G, dtype=np.float64)
    A = G.T @ G + lam * lam * np.eye(G.shape[1])
    return np.linalg.solve(A, G.T @ np.asarray(d, dtype=np.float64).ravel())


def dense_from_table(pr: dict, table: np.ndarray) -> np.ndarray:
    """Dense G of a spatially invariant kernel given by its entries per layer
    and cell offset (Sec. 2.1: an entry depends only on the offsets
    dx = p - pxl - i, dy = q - pyl - j and the layer r):
    G[j sx + i, r nx ny + q nx + p] = table[r][dy + sy - 1 + pyl][dx + sx - 1 + pxl]."""
    sx, sy, nz, pxl, pyl = pr["sx"], pr["sy"], pr["nz"], pr["pxl"], pr["pyl"]
    nx, ny = sx + pxl + pr["pxr"], sy + pyl + pr["pyr"]
    t = np.asarray(table, dtype=np.float64).reshape(nz, sy + ny - 1, sx + nx - 1)
    ix = (np.arange(nx)[None, :] - pxl - np.arange(sx)[:, None]) + sx - 1 + pxl     # [sx, nx]
    iy = (np.arange(ny)[None, :] - pyl - np.arange(sy)[:, None]) + sy - 1 + pyl     # [sy, ny]
    g = t[:, iy[:, None, :, None], ix[None, :, None, :]]                             # [nz, sy, sx, ny, nx]
    return np.ascontiguousarray(g.transpose(1, 2, 0, 3, 4).reshape(sy * sx, nz * ny * nx))
