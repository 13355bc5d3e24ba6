"""ctypes declarations of the C ABI in include/bttb.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
#: the in-tree build; BTTB_LIB selects another build of the same sources
LIB_PATH = os.environ.get("BTTB_LIB", os.path.join(_HERE, "libbttb.so"))

BTTB_OK = 0
STATUS_NAMES = {0: "BTTB_OK", 1: "BTTB_ERR_INVALID_VALUE", 2: "BTTB_ERR_NULL_POINTER",
                3: "BTTB_ERR_UNSUPPORTED", 4: "BTTB_ERR_WORKSPACE_TOO_SMALL", 5: "BTTB_ERR_HIP",
                6: "BTTB_ERR_INTERNAL", 7: "BTTB_ERR_OUT_OF_MEMORY"}
BTTB_GRAVITY_GZ, BTTB_MAGNETIC_TMI, BTTB_USER_TABLE, BTTB_HESSIAN, BTTB_PROBE = 0, 1, 2, 3, 99
BTTB_FP32, BTTB_FP64 = 0, 1
BTTB_ACC_DEFAULT, BTTB_ACC_PLAIN, BTTB_ACC_TWOSUM, BTTB_ACC_WIDE = 0, 1, 2, 3
BTTB_SPECTRUM_AUTO, BTTB_SPECTRUM_COMPLEX, BTTB_SPECTRUM_REAL_EVEN = 0, 1, 2
#: BTTB_NOALLOC_SCRATCH_BYTES: the device scratch array of bttb_forward_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20

#: every symbol include/bttb.h declares
EXPORTS = ["bttb_plan_create", "bttb_plan_destroy", "bttb_plan_query", "bttb_plan_memory_check", "bttb_kernel_generate",
           "bttb_forward", "bttb_transpose", "bttb_forward_noalloc", "bttb_forward_profiled",
           "bttb_transpose_profiled", "bttb_debug_generator", "bttb_debug_cap_grid", "bttb_plan_spectrum_form", "bttb_kernel_generate_table", "bttb_cgls_query", "bttb_cgls", "bttb_batch_create", "bttb_batch_query", "bttb_batch_run",
           "bttb_batch_destroy", "bttb_autotune_query", "bttb_autotune", "bttb_status_string",
           "bttb_last_error"]


class BatchIO(ctypes.Structure):
    _fields_ = [("spectra", ctypes.c_void_p), ("m", ctypes.c_void_p), ("d", ctypes.c_void_p),
                ("r", ctypes.c_void_p), ("mt", ctypes.c_void_p), ("nrhs", ctypes.c_int32)]


class ProblemDesc(ctypes.Structure):
    _fields_ = [
        ("problem", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("sx", ctypes.c_int32), ("sy", ctypes.c_int32),
        ("pxl", ctypes.c_int32), ("pxr", ctypes.c_int32), ("pyl", ctypes.c_int32), ("pyr", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("z_edges", ctypes.POINTER(ctypes.c_double)),
        ("station_height", ctypes.c_double),
        ("inclination_deg", ctypes.c_double), ("declination_deg", ctypes.c_double),
        ("field_nT", ctypes.c_double), ("scale", ctypes.c_double),
        ("nx_fft", ctypes.c_int32), ("ny_fft", ctypes.c_int32),
        ("accumulation", ctypes.c_int32), ("layer_chunk", ctypes.c_int32),
        ("row_tile", ctypes.c_int32), ("col_tile", ctypes.c_int32),
        ("spectrum_form", ctypes.c_int32),
        ("hessian", ctypes.c_double * 6),
    ]


class BttbError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        self.status = status
        super().__init__("%s failed: %s (%s)" % (fn, STATUS_NAMES.get(status, status), msg))


_handle = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libbttb.so; raises if it has not been built (no fallback exists)."""
    global _handle
    if _handle is not None:
        return _handle
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError("libbttb.so is not built (%s); run python -m paper_1912_06976_amd.build" % p)
    L = ctypes.CDLL(p)
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    L.bttb_plan_create.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(vp)]
    L.bttb_plan_destroy.argtypes = [vp]
    L.bttb_plan_query.argtypes = [vp, i32, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32)]
    L.bttb_plan_memory_check.argtypes = [vp, i32, sz, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.bttb_kernel_generate.argtypes = [vp, vp, vp, sz, vp]
    L.bttb_forward.argtypes = [vp, vp, vp, vp, i32, vp, sz, vp]
    L.bttb_transpose.argtypes = [vp, vp, vp, vp, i32, vp, sz, vp]
    L.bttb_forward_noalloc.argtypes = [vp, vp, vp, vp, i32, vp]
    L.bttb_forward_profiled.argtypes = [vp, vp, vp, vp, i32, vp, sz, vp, ctypes.POINTER(ctypes.c_float)]
    L.bttb_transpose_profiled.argtypes = [vp, vp, vp, vp, i32, vp, sz, vp, ctypes.POINTER(ctypes.c_float)]
    L.bttb_debug_generator.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), vp, sz, vp]
    L.bttb_debug_cap_grid.argtypes = [i32]
    L.bttb_plan_spectrum_form.argtypes = [vp, ctypes.POINTER(i32)]
    L.bttb_kernel_generate_table.argtypes = [vp, vp, vp, vp, sz, vp]
    L.bttb_cgls_query.argtypes = [vp, ctypes.POINTER(sz)]
    L.bttb_cgls.argtypes = [vp, vp, vp, vp, ctypes.c_double, i32, vp, vp, sz, vp]
    L.bttb_batch_create.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(vp)]
    L.bttb_batch_query.argtypes = [vp, ctypes.POINTER(sz)]
    L.bttb_batch_run.argtypes = [vp, ctypes.POINTER(BatchIO), vp, sz, vp]
    L.bttb_batch_destroy.argtypes = [vp]
    L.bttb_autotune_query.argtypes = [ctypes.POINTER(ProblemDesc), i32, ctypes.POINTER(sz)]
    L.bttb_autotune.argtypes = [ctypes.POINTER(ProblemDesc), i32, vp, sz, vp, ctypes.POINTER(ProblemDesc),
                                ctypes.POINTER(ctypes.c_float)]
    L.bttb_status_string.argtypes = [ctypes.c_int]
    L.bttb_status_string.restype = ctypes.c_char_p
    L.bttb_last_error.argtypes = []
    L.bttb_last_error.restype = ctypes.c_char_p
    for name in ["bttb_plan_create", "bttb_plan_destroy", "bttb_plan_query", "bttb_plan_memory_check",
                 "bttb_kernel_generate",
                 "bttb_forward", "bttb_transpose", "bttb_forward_noalloc", "bttb_forward_profiled",
                 "bttb_transpose_profiled", "bttb_debug_generator", "bttb_debug_cap_grid", "bttb_plan_spectrum_form", "bttb_kernel_generate_table", "bttb_cgls_query", "bttb_cgls", "bttb_batch_create", "bttb_batch_query", "bttb_batch_run",
                 "bttb_batch_destroy", "bttb_autotune_query", "bttb_autotune"]:
        getattr(L, name).restype = ctypes.c_int
    _handle = L
    return L


def check(fn: str, status: int):
    if status != BTTB_OK:
        msg = load().bttb_last_error().decode(errors="replace")
        raise BttbError(fn, status, msg)
