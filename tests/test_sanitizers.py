"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C source is rebuilt with gcc's sanitizers and exercised on
small problems; the host part of the HIP library (plans, queries, argument
checks, batch bookkeeping) is rebuilt with the sanitizers applied to host
code only, linked with the regular kernel objects, and runs the C-ABI host
tests.  Every case runs in a child process with the sanitizer runtime
preloaded, and any report ends it with an error."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_runtime(name):
    try:
        p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    except OSError:
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _run_child(code_or_args, env_extra, timeout=900):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    args = [sys.executable] + (["-c", code_or_args] if isinstance(code_or_args, str) else code_or_args)
    return subprocess.run(args, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)


ORACLE_CALLS = r"""
import sys
sys.path[:0] = ['tests', '.']
import numpy as np
import workloads as W
import oracle
from _common import oracle_problem
probs = [W.small_gravity(), W.magnetic_24(),
         W.problem(W.MAGNETIC, 7, 5, 3, 2, 0, 1, 3, dx=25.0, dy=40.0, z_edges=[0, 10, 25, 45], h=12.5,
                   incl=35.0, decl=70.0, field_nT=45000.0),
         W.problem(W.PROBE, 5, 4, 3, 2, 1, 1, 2, dx=25.0, dy=50.0, dz=10.0)]
for pr in probs:
    P = oracle_problem(pr)
    G = oracle.dense_G(P)
    Gq, A = oracle.dense_G_quad(P, with_abs=True)
    t, a = oracle.offset_table_quad(P)
    nx, ny, nz = W.dims(pr)
    m = W.normal_model(pr, 1)
    r = W.normal_data(pr, 2)
    st = [(0, 0), (pr["sx"] - 1, pr["sy"] - 1)]
    pq = np.array([[0, 0, 0], [nx - 1, ny - 1, nz - 1]])
    ds = oracle.station_sums(P, m, st)
    ts = oracle.prism_sums(P, r, pq)
    ref = G @ m.ravel()
    assert np.allclose(ds, [ref[j * pr["sx"] + i] for i, j in st], rtol=1e-9, atol=1e-300)
print("oracle ok")
"""


def test_oracle_under_sanitizers(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not available")
    lib = str(tmp_path / "prism_oracle_san.so")
    src = os.path.join(ROOT, "oracle", "prism_oracle.c")
    cmd = ["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
           "-shared", "-fPIC", "-o", lib, src, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True, cwd=os.path.join(ROOT, "oracle"))
    r = _run_child(ORACLE_CALLS, {"LD_PRELOAD": asan, "ORACLE_LIB": lib})
    assert r.returncode == 0 and "oracle ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]


def _clang_asan_runtime():
    base = "/opt/rocm/lib/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for v in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def test_host_library_under_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1912_06976_amd import build as B
    rt = _clang_asan_runtime()
    kernel_objs = [os.path.join(B.BUILD, os.path.splitext(n)[0] + ".o") for n in B.KERNEL_SOURCES]
    if rt is None or not all(os.path.exists(o) for o in kernel_objs):
        pytest.skip("needs the clang AddressSanitizer runtime and a built library (__graft_entry__.build())")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in ("bttb_host.hip", "bttb_cgls.hip"):
        obj = str(tmp_path / (src + ".o"))
        cmd = [B.HIPCC, *B.FLAGS, "-O1", "-g", *san, "-c", os.path.join(B.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    lib = str(tmp_path / "libbttb_san.so")
    cmd = [B.HIPCC, "--offload-arch=" + B.ARCH, "-shared", "-fPIC", *san, "-o", lib, *objs, *kernel_objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = _run_child(["-m", "pytest", "tests/test_abi_host.py", "-x", "-q", "-p", "no:cacheprovider"],
                   {"LD_PRELOAD": rt, "BTTB_LIB": lib})
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
