"""Fast BTTB forward / transpose products with 3-D gravity and magnetic kernels
on AMD Instinct MI355X (gfx950).

The products d = G m and G^T r of Hogue, Renaut & Vatankhah (arXiv
1912.06976) run in hand-written HIP kernels behind the C ABI of
``include/bttb.h`` (libbttb.so); this package is its Python binding.
"""
from ._lib import BttbError, EXPORTS, LIB_PATH, load  # noqa: F401
from .plan import (Batch, Plan, bttb_batch_create, bttb_batch_destroy, bttb_batch_query,  # noqa: F401
                   bttb_autotune, bttb_batch_run, bttb_debug_cap_grid, bttb_debug_generator, bttb_forward, bttb_forward_noalloc,  # noqa: F401
                   bttb_forward_profiled,
                   bttb_plan_spectrum_form, bttb_cgls, bttb_cgls_query, bttb_kernel_generate_table,
                   bttb_kernel_generate, bttb_plan_create, bttb_plan_destroy, bttb_plan_query, bttb_plan_memory_check,
                   bttb_transpose, bttb_transpose_profiled, hessian_weights_component,
                   hessian_weights_tmi)

from .autograd import BTTBForward, BTTBTranspose, bttb_matvec, bttb_rmatvec  # noqa: F401

__all__ = ["Plan", "Batch", "bttb_autotune", "bttb_batch_create", "bttb_batch_query", "bttb_batch_run",
           "bttb_batch_destroy", "BTTBForward", "BTTBTranspose", "bttb_matvec", "bttb_rmatvec", "BttbError", "bttb_plan_create", "bttb_plan_destroy", "bttb_plan_query", "bttb_plan_memory_check",
           "bttb_kernel_generate", "bttb_forward", "bttb_forward_noalloc", "bttb_transpose", "bttb_forward_profiled",
           "bttb_transpose_profiled", "bttb_debug_cap_grid", "bttb_debug_generator", "bttb_plan_spectrum_form", "bttb_cgls", "bttb_cgls_query", "bttb_kernel_generate_table", "hessian_weights_component",
           "hessian_weights_tmi", "load"]
