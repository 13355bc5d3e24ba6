"""Build libbttb.so (gfx950) in-tree with hipcc.

    python -m paper_1912_06976_amd.build

Compiles every HIP translation unit under csrc/ for gfx950 (in parallel,
longest first) and links them into
paper_1912_06976_amd/libbttb.so.  Packed FP32 instructions are disabled
(-packed-fp32-ops): the compiler must emit scalar-lane FP32 arithmetic only.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.environ.get("BTTB_LIB_OUT", os.path.join(HERE, "libbttb.so"))
BUILD = os.environ.get("BTTB_BUILD_DIR", os.path.join(ROOT, "_build"))
# kernels and their dispatch; the row and column kernels are instantiated per
# group of transform lengths (bttb_rows_*.hip, bttb_cols_*.hip) so that the
# translation units compile in parallel
KERNEL_SOURCES = ["bttb_cols_d.hip", "bttb_rows_d.hip", "bttb_cols_c.hip", "bttb_rows_c.hip",
                  "bttb_cols_b.hip", "bttb_rows_b.hip", "bttb_cols_a.hip", "bttb_rows_a.hip",
                  "bttb_kernels.hip", "bttb_cols.hip"]
SOURCES = KERNEL_SOURCES + ["bttb_cgls.hip", "bttb_host.hip"]
JOBS = int(os.environ.get("BTTB_BUILD_JOBS", str(min(len(SOURCES), os.cpu_count() or 4))))

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("BTTB_ARCH", "gfx950")
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I" + os.path.join(ROOT, "include"),
         *os.environ.get("BTTB_EXTRA_FLAGS", "").split()]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on " + src)
    return obj


def build(verbose: bool = False) -> str:
    """Compile all sources (always) and link libbttb.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, JOBS)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
