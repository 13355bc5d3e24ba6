"""Python binding of libbttb.so with the C ABI's names.

Every function marshals torch tensors (device memory) and torch's current
HIP stream into the C entry points of include/bttb.h; all computation runs in
the library's HIP kernels.  There is no fallback path: if libbttb.so is
missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import check

_KIND = {"gravity": _lib.BTTB_GRAVITY_GZ, "magnetic": _lib.BTTB_MAGNETIC_TMI, "table": _lib.BTTB_USER_TABLE,
         "hessian": _lib.BTTB_HESSIAN, "probe": _lib.BTTB_PROBE}
_PREC = {"fp32": _lib.BTTB_FP32, "fp64": _lib.BTTB_FP64}
_FORM = {"auto": _lib.BTTB_SPECTRUM_AUTO, "complex": _lib.BTTB_SPECTRUM_COMPLEX,
         "real_even": _lib.BTTB_SPECTRUM_REAL_EVEN}
_ACC = {"default": _lib.BTTB_ACC_DEFAULT, "plain": _lib.BTTB_ACC_PLAIN, "twosum": _lib.BTTB_ACC_TWOSUM,
        "wide": _lib.BTTB_ACC_WIDE}


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _stream_obj(stream):
    return torch.cuda.current_stream() if stream is None else stream


def _capturing(s, is_current: bool) -> bool:
    """Whether stream s is being captured into a graph."""
    if is_current:
        return torch.cuda.is_current_stream_capturing()
    with torch.cuda.stream(s):
        return torch.cuda.is_current_stream_capturing()


def _empty_on(s, is_current: bool, shape, dtype, device) -> torch.Tensor:
    """torch.empty allocated on stream s (s is torch's current stream when
    is_current: no stream switch needed)."""
    if is_current:
        return torch.empty(shape, dtype=dtype, device=device)
    with torch.cuda.stream(s):
        return torch.empty(shape, dtype=dtype, device=device)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(int(t.data_ptr()))


def make_desc(problem: dict, precision: str = "fp32", accumulation: str = "default"):
    """Build the C descriptor from a problem dict (see workloads.problem)."""
    z = problem.get("z_edges")
    keep = None
    zp = None
    if z is not None:
        keep = np.ascontiguousarray(z, dtype=np.float64)
        zp = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d = _lib.ProblemDesc(
        problem=_KIND[problem["kind"]], precision=_PREC[precision],
        nx=0, ny=0, nz=problem["nz"], sx=problem["sx"], sy=problem["sy"],
        pxl=problem.get("pxl", 0), pxr=problem.get("pxr", 0), pyl=problem.get("pyl", 0),
        pyr=problem.get("pyr", 0), dx=problem["dx"], dy=problem["dy"], dz=problem.get("dz", 0.0),
        z_edges=zp, station_height=problem.get("h", 0.0),
        inclination_deg=problem.get("incl", 90.0), declination_deg=problem.get("decl", 0.0),
        field_nT=problem.get("field_nT", 50000.0), scale=problem.get("scale", 0.0),
        nx_fft=problem.get("nx_fft", 0), ny_fft=problem.get("ny_fft", 0),
        accumulation=_ACC[accumulation], layer_chunk=problem.get("layer_chunk", 0),
        row_tile=problem.get("row_tile", 0), col_tile=problem.get("col_tile", 0),
        spectrum_form=_FORM[problem.get("spectrum_form", "auto")],
        hessian=(ctypes.c_double * 6)(*[float(v) for v in (problem.get("hessian") or (0.0,) * 6)]))
    return d, keep


def _unit(incl_deg: float, decl_deg: float):
    i, d = math.radians(incl_deg), math.radians(decl_deg)
    return (math.cos(i) * math.cos(d), math.cos(i) * math.sin(d), math.sin(i))


def hessian_weights_tmi(incl: float, decl: float, m_incl: float, m_decl: float):
    """Weights (w_xx, w_yy, w_zz, w_xy, w_xz, w_yz) of a "hessian" kernel for
    the total-field anomaly f^T U m of a magnetisation of direction (m_incl,
    m_decl) in a field of direction (incl, decl) (x North, y East, z down):
    w_aa = f_a m_a, w_ab = f_a m_b + f_b m_a."""
    f, m = _unit(incl, decl), _unit(m_incl, m_decl)
    return (f[0] * m[0], f[1] * m[1], f[2] * m[2], f[0] * m[1] + f[1] * m[0],
            f[0] * m[2] + f[2] * m[0], f[1] * m[2] + f[2] * m[1])


def hessian_weights_component(a: str, b: str):
    """Weights selecting one component U_ab (a, b in "xyz"), e.g. ("z", "z")
    for the gravity gradient g_zz."""
    key = "".join(sorted(a + b))
    order = ["xx", "yy", "zz", "xy", "xz", "yz"]
    return tuple(1.0 if k == key else 0.0 for k in order)


def bttb_plan_create(problem: dict, precision: str = "fp32", accumulation: str = "default") -> int:
    L = _lib.load()
    d, keep = make_desc(problem, precision, accumulation)
    h = ctypes.c_void_p()
    check("bttb_plan_create", L.bttb_plan_create(ctypes.byref(d), ctypes.byref(h)))
    del keep
    return h.value


def bttb_plan_destroy(plan: int) -> None:
    check("bttb_plan_destroy", _lib.load().bttb_plan_destroy(ctypes.c_void_p(plan)))


def bttb_plan_query(plan: int, nrhs: int = 1):
    """Returns (spectra_bytes, workspace_bytes, nx_fft, ny_fft)."""
    sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    nx, ny = ctypes.c_int32(), ctypes.c_int32()
    check("bttb_plan_query", _lib.load().bttb_plan_query(ctypes.c_void_p(plan), nrhs, ctypes.byref(sb),
                                                          ctypes.byref(wb), ctypes.byref(nx),
                                                          ctypes.byref(ny)))
    return sb.value, wb.value, nx.value, ny.value


def bttb_plan_memory_check(plan: int, nrhs: int = 1, available: int = 0):
    """The memory guard: returns (need_bytes, available_bytes) for the plan's
    spectra, workspace and one product's input and output with nrhs
    right-hand sides; available = 0 compares against the current device's
    free memory.  Raises BttbError (BTTB_ERR_OUT_OF_MEMORY) when they do not fit."""
    need, avail = ctypes.c_size_t(), ctypes.c_size_t()
    check("bttb_plan_memory_check",
          _lib.load().bttb_plan_memory_check(ctypes.c_void_p(plan), nrhs, int(available), ctypes.byref(need),
                                             ctypes.byref(avail)))
    return need.value, avail.value


def bttb_plan_spectrum_form(plan: int) -> str:
    """The plan's stored spectrum form: "complex" or "real_even"."""
    f = ctypes.c_int32()
    check("bttb_plan_spectrum_form", _lib.load().bttb_plan_spectrum_form(ctypes.c_void_p(plan), ctypes.byref(f)))
    return {v: k for k, v in _FORM.items()}[f.value]


def bttb_kernel_generate(plan: int, spectra: torch.Tensor, workspace: torch.Tensor, stream=None) -> None:
    check("bttb_kernel_generate",
          _lib.load().bttb_kernel_generate(ctypes.c_void_p(plan), _ptr(spectra), _ptr(workspace),
                                           workspace.numel() * workspace.element_size(),
                                           _stream_ptr(stream)))


def bttb_kernel_generate_table(plan: int, table: torch.Tensor, spectra: torch.Tensor, workspace: torch.Tensor,
                               stream=None) -> None:
    """Spectra of a "table" plan from the caller's entries: table is a
    contiguous float64 device tensor [nz, sy + ny - 1, sx + nx - 1] indexed by
    the cell offsets (dy + sy - 1 + pyl, dx + sx - 1 + pxl)."""
    if table.device.type != "cuda" or table.dtype != torch.float64 or not table.is_contiguous():
        raise ValueError("table must be a contiguous float64 CUDA tensor")
    check("bttb_kernel_generate_table",
          _lib.load().bttb_kernel_generate_table(ctypes.c_void_p(plan), _ptr(table), _ptr(spectra), _ptr(workspace),
                                                 workspace.numel() * workspace.element_size(),
                                                 _stream_ptr(stream)))


def bttb_forward(plan: int, spectra: torch.Tensor, m: torch.Tensor, d: torch.Tensor, nrhs: int,
                 workspace: torch.Tensor, stream=None) -> None:
    check("bttb_forward",
          _lib.load().bttb_forward(ctypes.c_void_p(plan), _ptr(spectra), _ptr(m), _ptr(d), nrhs,
                                   _ptr(workspace), workspace.numel() * workspace.element_size(),
                                   _stream_ptr(stream)))


def bttb_forward_noalloc(plan: int, spectra: torch.Tensor, m: torch.Tensor, d: torch.Tensor, nrhs: int,
                         stream=None) -> None:
    """bttb_forward with the library's own device scratch array as workspace
    (no allocation; calls on one GPU must not overlap)."""
    check("bttb_forward_noalloc",
          _lib.load().bttb_forward_noalloc(ctypes.c_void_p(plan), _ptr(spectra), _ptr(m), _ptr(d), nrhs,
                                           _stream_ptr(stream)))


def bttb_transpose(plan: int, spectra: torch.Tensor, r: torch.Tensor, mt: torch.Tensor, nrhs: int,
                   workspace: torch.Tensor, stream=None) -> None:
    check("bttb_transpose",
          _lib.load().bttb_transpose(ctypes.c_void_p(plan), _ptr(spectra), _ptr(r), _ptr(mt), nrhs,
                                     _ptr(workspace), workspace.numel() * workspace.element_size(),
                                     _stream_ptr(stream)))


def _profiled(fn: str, plan, spectra, x, y, nrhs, workspace, stream):
    ms = (ctypes.c_float * 3)()
    check(fn, getattr(_lib.load(), fn)(ctypes.c_void_p(plan), _ptr(spectra), _ptr(x), _ptr(y), nrhs,
                                       _ptr(workspace), workspace.numel() * workspace.element_size(),
                                       _stream_ptr(stream), ms))
    return [float(v) for v in ms]


def bttb_forward_profiled(plan: int, spectra, m, d, nrhs: int, workspace, stream=None):
    """bttb_forward with per-kernel HIP-event timing; returns the 3 kernel times [ms]."""
    return _profiled("bttb_forward_profiled", plan, spectra, m, d, nrhs, workspace, stream)


def bttb_transpose_profiled(plan: int, spectra, r, mt, nrhs: int, workspace, stream=None):
    """bttb_transpose with per-kernel HIP-event timing; returns the 3 kernel times [ms]."""
    return _profiled("bttb_transpose_profiled", plan, spectra, r, mt, nrhs, workspace, stream)


def bttb_cgls_query(plan: int) -> int:
    """Workspace bytes of bttb_cgls for this plan."""
    sz = ctypes.c_size_t()
    check("bttb_cgls_query", _lib.load().bttb_cgls_query(ctypes.c_void_p(plan), ctypes.byref(sz)))
    return sz.value


def bttb_cgls(plan: int, spectra: torch.Tensor, d: torch.Tensor, m: torch.Tensor, lam: float, iterations: int,
              history: torch.Tensor | None, workspace: torch.Tensor, stream=None) -> None:
    """CGLS for min ||G m - d||^2 + lam^2 ||m||^2, m updated in place; history
    (optional, float64 [iterations + 1, 3]) receives (||r||^2, ||m||^2, ||s||^2)."""
    hp = _ptr(history) if history is not None else ctypes.c_void_p(0)
    check("bttb_cgls",
          _lib.load().bttb_cgls(ctypes.c_void_p(plan), _ptr(spectra), _ptr(d), _ptr(m), float(lam), int(iterations),
                                hp, _ptr(workspace), workspace.numel() * workspace.element_size(),
                                _stream_ptr(stream)))


def bttb_debug_cap_grid(max_blocks: int) -> None:
    check("bttb_debug_cap_grid", _lib.load().bttb_debug_cap_grid(max_blocks))


def bttb_debug_generator(plan: int, layer: int, workspace: torch.Tensor, stream=None) -> np.ndarray:
    _, _, nx, ny = bttb_plan_query(plan, 1)
    out = np.empty((ny, nx), dtype=np.float64)
    check("bttb_debug_generator",
          _lib.load().bttb_debug_generator(ctypes.c_void_p(plan), layer,
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           _ptr(workspace), workspace.numel() * workspace.element_size(),
                                           _stream_ptr(stream)))
    return out


class Plan:
    """A plan plus its spectra, on one device.

    ``Plan(problem, precision)`` validates the problem (host only);
    ``generate()`` allocates the spectra and fills them on the GPU;
    ``forward(m)`` / ``transpose(r)`` run the products on torch's current stream
    (or the ``stream`` argument).  Each stream gets its own cached workspace,
    allocated on that stream, and default outputs are allocated on the stream
    the product runs on, so products of one plan may run on several streams.
    """

    def __init__(self, problem: dict, precision: str = "fp32", accumulation: str = "default",
                 device="cuda"):
        self.problem = dict(problem)
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.device = torch.device(device)
        self.handle = bttb_plan_create(problem, precision, accumulation)
        self.spectra_bytes, self._ws1, self.nx_fft, self.ny_fft = bttb_plan_query(self.handle, 1)
        self.spectrum_form = bttb_plan_spectrum_form(self.handle)
        self.sx, self.sy, self.nz = problem["sx"], problem["sy"], problem["nz"]
        self.nx = self.sx + problem.get("pxl", 0) + problem.get("pxr", 0)
        self.ny = self.sy + problem.get("pyl", 0) + problem.get("pyr", 0)
        self.spectra = None
        self._ws = {}          # cached workspace per stream (keyed by the HIP stream handle)
        self._ws_bytes = {}    # workspace bytes per right-hand-side count

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                bttb_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    # -- memory -----------------------------------------------------------
    def workspace_bytes(self, nrhs: int = 1) -> int:
        b = self._ws_bytes.get(nrhs)
        if b is None:
            b = self._ws_bytes[nrhs] = bttb_plan_query(self.handle, nrhs)[1]
        return b

    def workspace(self, nrhs: int = 1, stream=None) -> torch.Tensor:
        """The workspace of products with nrhs right-hand sides on `stream`
        (default: the current stream), cached per stream and allocated on it:
        a larger replacement frees the old block on the same stream, after
        the products already queued there.  During graph capture a fresh,
        uncached workspace comes from the graph's memory pool."""
        return self._workspace(nrhs, _stream_obj(stream), stream is None)

    def _workspace(self, nrhs: int, s, is_current: bool) -> torch.Tensor:
        key = int(s.cuda_stream)
        need = self.workspace_bytes(nrhs)
        if _capturing(s, is_current):
            # under graph capture: a workspace of the graph's own memory pool,
            # not cached (it must not be reused outside the graph)
            with torch.cuda.stream(s):
                return torch.empty(need, dtype=torch.uint8, device=self.device)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            self._ws.pop(key, None)
            with torch.cuda.stream(s):
                ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    # -- operations ---------------------------------------------------------
    def generate(self, table: torch.Tensor | None = None, stream=None) -> "Plan":
        """Fill the spectra: from the closed-form kernel, or (a "table" plan)
        from the caller's entries, [nz, sy + ny - 1, sx + nx - 1] float64 on
        the device, indexed by the cell offsets."""
        if self.spectra is None:
            with torch.cuda.device(self.device):
                bttb_plan_memory_check(self.handle, 1)
            self.spectra = torch.empty(self.spectra_bytes, dtype=torch.uint8, device=self.device)
        if self.problem["kind"] == "table":
            if table is None:
                raise ValueError("a table plan needs its entries: generate(table=...)")
            want = (self.nz, self.sy + self.ny - 1, self.sx + self.nx - 1)
            if tuple(table.shape) != want:
                raise ValueError("table has shape %s, expected %s" % (tuple(table.shape), want))
            bttb_kernel_generate_table(self.handle, table.contiguous(), self.spectra, self.workspace(1, stream),
                                       stream)
        else:
            bttb_kernel_generate(self.handle, self.spectra, self.workspace(1, stream), stream)
        return self

    def _check_vec(self, t: torch.Tensor, tail, name):
        if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s CUDA tensor" % (name, self.dtype))
        if tuple(t.shape[-len(tail):]) != tuple(tail):
            raise ValueError("%s has shape %s, expected [..., %s]" % (name, tuple(t.shape), tail))
        return int(math.prod(t.shape[:-len(tail)]))

    def forward(self, m: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if self.spectra is None:
            raise RuntimeError("call generate() first")
        nrhs = self._check_vec(m, (self.nz, self.ny, self.nx), "m")
        s = _stream_obj(stream)
        if out is None:
            out = _empty_on(s, stream is None, m.shape[:-3] + (self.sy, self.sx), self.dtype, m.device)
        if self._check_vec(out, (self.sy, self.sx), "out") != nrhs:
            raise ValueError("out holds a different number of right-hand sides than m")
        if nrhs == 0:
            return out
        bttb_forward(self.handle, self.spectra, m, out, nrhs, self._workspace(nrhs, s, stream is None), s)
        return out

    def transpose(self, r: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if self.spectra is None:
            raise RuntimeError("call generate() first")
        nrhs = self._check_vec(r, (self.sy, self.sx), "r")
        s = _stream_obj(stream)
        if out is None:
            out = _empty_on(s, stream is None, r.shape[:-2] + (self.nz, self.ny, self.nx), self.dtype, r.device)
        if self._check_vec(out, (self.nz, self.ny, self.nx), "out") != nrhs:
            raise ValueError("out holds a different number of right-hand sides than r")
        if nrhs == 0:
            return out
        bttb_transpose(self.handle, self.spectra, r, out, nrhs, self._workspace(nrhs, s, stream is None), s)
        return out

    def cgls(self, d: torch.Tensor, lam: float, iterations: int, m0: torch.Tensor | None = None, stream=None):
        """Regularised least squares min ||G m - d||^2 + lam^2 ||m||^2 by CGLS on
        the device (one forward and one transpose product per step).  Returns
        (m, history) with history a float64 tensor [iterations + 1, 3] of
        (||r||^2, ||m||^2, ||s||^2)."""
        if self.spectra is None:
            raise RuntimeError("call generate() first")
        self._check_vec(d, (self.sy, self.sx), "d")
        if d.dim() != 2:
            raise ValueError("d must be [sy, sx] (one right-hand side)")
        if m0 is not None:
            self._check_vec(m0, (self.nz, self.ny, self.nx), "m0")
        with torch.cuda.stream(_stream_obj(stream)):
            if m0 is None:
                m = torch.zeros((self.nz, self.ny, self.nx), dtype=self.dtype, device=d.device)
            else:
                m = m0.clone()
            hist = torch.zeros((iterations + 1, 3), dtype=torch.float64, device=d.device)
            ws = torch.empty(bttb_cgls_query(self.handle), dtype=torch.uint8, device=d.device)
        bttb_cgls(self.handle, self.spectra, d, m, lam, iterations, hist, ws, stream)
        return m, hist

    def debug_generator(self, layer: int) -> np.ndarray:
        return bttb_debug_generator(self.handle, layer, self.workspace(1), None)


def bttb_batch_create(plans, max_nrhs: int = 1) -> int:
    arr = (ctypes.c_void_p * len(plans))(*[p.handle if isinstance(p, Plan) else p for p in plans])
    h = ctypes.c_void_p()
    check("bttb_batch_create", _lib.load().bttb_batch_create(arr, len(plans), max_nrhs, ctypes.byref(h)))
    return h.value


def bttb_batch_query(batch: int) -> int:
    wb = ctypes.c_size_t()
    check("bttb_batch_query", _lib.load().bttb_batch_query(ctypes.c_void_p(batch), ctypes.byref(wb)))
    return wb.value


def bttb_batch_run(batch: int, io, workspace: torch.Tensor, stream=None) -> None:
    arr = (_lib.BatchIO * len(io))(*io)
    check("bttb_batch_run", _lib.load().bttb_batch_run(ctypes.c_void_p(batch), arr, _ptr(workspace),
                                                       workspace.numel() * workspace.element_size(),
                                                       _stream_ptr(stream)))


def bttb_batch_destroy(batch: int) -> None:
    check("bttb_batch_destroy", _lib.load().bttb_batch_destroy(ctypes.c_void_p(batch)))


class Batch:
    """Many generated plans of one precision run together as one graph launch.

    ``run(ms=..., rs=...)`` takes, per plan, a model tensor (or None) for the
    forward product and a data tensor (or None) for the transpose product and
    returns the lists of outputs.  The plans must stay alive.
    """

    def __init__(self, plans, max_nrhs: int = 1):
        self.plans = list(plans)
        for p in self.plans:
            if p.spectra is None:
                raise RuntimeError("generate() every plan before batching it")
        self.max_nrhs = max_nrhs
        self.handle = bttb_batch_create(self.plans, max_nrhs)
        self.workspace = torch.empty(bttb_batch_query(self.handle), dtype=torch.uint8,
                                     device=self.plans[0].device)
        self._outs = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                bttb_batch_destroy(h)
            except Exception:
                pass
            self.handle = None

    def run(self, ms=None, rs=None, stream=None, out_ds=None, out_mts=None):
        """Outputs are new tensors unless out_ds / out_mts (lists matching ms /
        rs) are given; with the same input and output tensors every call
        replays the captured graph."""
        n = len(self.plans)
        ms = list(ms) if ms is not None else [None] * n
        rs = list(rs) if rs is not None else [None] * n
        out_ds = list(out_ds) if out_ds is not None else [None] * n
        out_mts = list(out_mts) if out_mts is not None else [None] * n
        io, ds, mts = [], [], []
        for p, m, r, od, omt in zip(self.plans, ms, rs, out_ds, out_mts):
            nr = 1
            d = mt = None
            if m is not None:
                nr = p._check_vec(m, (p.nz, p.ny, p.nx), "m")
                d = od if od is not None else torch.empty(m.shape[:-3] + (p.sy, p.sx), dtype=p.dtype, device=m.device)
                if p._check_vec(d, (p.sy, p.sx), "d") != nr:
                    raise ValueError("output d has the wrong number of right-hand sides")
            if r is not None:
                nr2 = p._check_vec(r, (p.sy, p.sx), "r")
                if m is not None and nr2 != nr:
                    raise ValueError("m and r of one problem need the same number of right-hand sides")
                nr = nr2
                mt = omt if omt is not None else torch.empty(r.shape[:-2] + (p.nz, p.ny, p.nx), dtype=p.dtype,
                                                             device=r.device)
                if p._check_vec(mt, (p.nz, p.ny, p.nx), "mt") != nr:
                    raise ValueError("output mt has the wrong number of right-hand sides")
            io.append(_lib.BatchIO(p.spectra.data_ptr(), m.data_ptr() if m is not None else None,
                                   d.data_ptr() if d is not None else None,
                                   r.data_ptr() if r is not None else None,
                                   mt.data_ptr() if mt is not None else None, nr))
            ds.append(d)
            mts.append(mt)
        bttb_batch_run(self.handle, io, self.workspace, stream)
        return ds, mts


def bttb_autotune(problem: dict, precision: str = "fp32", nrhs: int = 1, accumulation: str = "default",
                  stream=None):
    """Time the candidate configurations for this problem on the current
    device (or read them from the on-disk cache) and return (problem dict with
    nx_fft / ny_fft / layer_chunk / row_tile / col_tile filled in, ms per
    forward + transpose pair)."""
    L = _lib.load()
    d, keep = make_desc(problem, precision, accumulation)
    sb = ctypes.c_size_t()
    check("bttb_autotune_query", L.bttb_autotune_query(ctypes.byref(d), nrhs, ctypes.byref(sb)))
    scratch = torch.empty(sb.value, dtype=torch.uint8, device="cuda")
    out = _lib.ProblemDesc()
    ms = ctypes.c_float()
    check("bttb_autotune", L.bttb_autotune(ctypes.byref(d), nrhs, _ptr(scratch), sb.value, _stream_ptr(stream),
                                           ctypes.byref(out), ctypes.byref(ms)))
    del keep, scratch
    tuned = dict(problem)
    tuned.update(layer_chunk=out.layer_chunk, row_tile=out.row_tile, col_tile=out.col_tile,
                 nx_fft=out.nx_fft, ny_fft=out.ny_fft)
    return tuned, ms.value
