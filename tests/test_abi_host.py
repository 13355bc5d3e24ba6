"""Host-side tests of the C ABI (no GPU needed): the library loads, exports
every symbol include/bttb.h declares, validates descriptors and reports
sizes.  No call here launches a kernel."""
import ctypes
import os
import re
import subprocess

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1912_06976_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1912_06976_amd import build
        build.build()
    return _lib.load()


def header_functions():
    txt = open(os.path.join(ROOT, "include", "bttb.h")).read()
    return sorted(set(re.findall(r"^\s*(?:bttb_status|const char\*)\s+(bttb_\w+)\(", txt, re.M)))


def test_exports_every_declared_symbol(lib):
    from paper_1912_06976_amd import _lib
    names = header_functions()
    assert set(names) == set(_lib.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)


def test_status_strings(lib):
    for code, name in [(0, "BTTB_OK"), (1, "BTTB_ERR_INVALID_VALUE"), (4, "BTTB_ERR_WORKSPACE_TOO_SMALL"),
                       (7, "BTTB_ERR_OUT_OF_MEMORY")]:
        assert lib.bttb_status_string(code).decode() == name


def _create(prob, prec="fp32", **over):
    from paper_1912_06976_amd.plan import make_desc
    from paper_1912_06976_amd import _lib
    d, keep = make_desc(prob, prec)
    for k, v in over.items():
        setattr(d, k, v)
    h = ctypes.c_void_p()
    st = _lib.load().bttb_plan_create(ctypes.byref(d), ctypes.byref(h))
    return st, h, _lib.load().bttb_last_error().decode()


@pytest.mark.parametrize("field,value,status", [
    ("sx", 0, 1), ("sy", -3, 1), ("nz", 0, 1), ("pxl", -1, 1), ("dx", 0.0, 1), ("dy", float("nan"), 1),
    ("dz", -1.0, 1), ("station_height", -1.0, 1), ("problem", 7, 1), ("problem", 4, 1), ("precision", 3, 1),
    ("nx", 17, 1), ("nx_fft", 16, 1), ("nx_fft", 100, 3), ("nx_fft", 432, 3), ("ny_fft", 8192, 3), ("accumulation", 9, 1),
    ("layer_chunk", -1, 1), ("row_tile", 3, 1), ("col_tile", 4, 1), ("spectrum_form", 3, 1),
])
def test_invalid_descriptors_rejected(lib, field, value, status):
    st, h, msg = _create(W.small_gravity(), **{field: value})
    assert st == status and h.value is None and msg


def test_magnetic_field_checks(lib):
    st, _, _ = _create(W.magnetic_48x56(), inclination_deg=91.0)
    assert st == 1
    st, _, _ = _create(W.magnetic_48x56(), field_nT=0.0)
    assert st == 1
    st, h, _ = _create(W.magnetic_48x56())
    assert st == 0
    lib.bttb_plan_destroy(h)


def test_z_edges_validation(lib):
    pr = dict(W.small_gravity(), z_edges=[0.0, 10.0, 5.0, 20.0, 30.0, 40.0, 50.0, 60.0, 70.0])
    st, _, msg = _create(pr)
    assert st == 1 and "increasing" in msg
    pr = dict(W.small_gravity(), z_edges=[0.0, 10.0, 15.0, 20.0, 30.0, 40.0, 50.0, 60.0, 70.0])
    st, h, _ = _create(pr)
    assert st == 0
    lib.bttb_plan_destroy(h)


def test_null_pointers(lib):
    from paper_1912_06976_amd import _lib
    h = ctypes.c_void_p()
    assert lib.bttb_plan_create(None, ctypes.byref(h)) == 2
    assert lib.bttb_plan_query(None, 1, None, None, None, None) == 2
    assert lib.bttb_forward(None, None, None, None, 1, None, 0, None) == 2
    assert lib.bttb_transpose(None, None, None, None, 1, None, 0, None) == 2
    assert lib.bttb_kernel_generate(None, None, None, 0, None) == 2
    assert lib.bttb_plan_destroy(None) == 0


def test_sizes_and_fft_choice(lib):
    import paper_1912_06976_amd as B
    h = B.bttb_plan_create(dict(W.gravity_1024(), spectrum_form="complex"), "fp32")
    sb, wb, nx, ny = B.bttb_plan_query(h, 1)
    assert (nx, ny) == (2048, 2048)       # smallest power of two >= 1000 + 1024 - 1
    # spectra: 128 layers x 1024 packed columns x 2048 complex64, plus twiddle tables
    assert 128 * 2048 * 1024 * 8 <= sb <= 128 * 2048 * 1024 * 8 + 4 * 2048 * 16 + 4096
    assert B.bttb_plan_spectrum_form(h) == "complex"
    B.bttb_plan_destroy(h)
    # real even form (default for gravity): 128 layers x 1025 lines x 1025
    # FP32 values (line stride rounded up to 1056), plus twiddle tables
    h = B.bttb_plan_create(W.gravity_1024(), "fp32")
    sb, wb, nx, ny = B.bttb_plan_query(h, 1)
    assert B.bttb_plan_spectrum_form(h) == "real_even"
    assert 128 * 1025 * 1056 * 4 <= sb <= 128 * 1025 * 1056 * 4 + 4 * 2048 * 16 + 4096
    sb4, wb4, _, _ = B.bttb_plan_query(h, 4)
    assert sb4 == sb and wb4 > wb
    with pytest.raises(B.BttbError):
        B.bttb_plan_query(h, 0)
    B.bttb_plan_destroy(h)
    h = B.bttb_plan_create(W.small_gravity(), "fp64")
    assert B.bttb_plan_query(h, 1)[2:] == (32, 32)
    B.bttb_plan_destroy(h)
    h = B.bttb_plan_create(dict(W.small_gravity(), nx_fft=64, ny_fft=128), "fp64")
    assert B.bttb_plan_query(h, 1)[2:] == (64, 128)
    B.bttb_plan_destroy(h)


def test_memory_guard_against_a_budget(lib):
    """The memory check with a caller's budget (no device query): the need is
    spectra + workspace + one input and output, each rounded to 256 bytes;
    a budget one byte short is refused with OUT_OF_MEMORY, the exact budget
    passes, and both figures come back either way."""
    import paper_1912_06976_amd as B
    from paper_1912_06976_amd import _lib
    up = lambda b: (b + 255) // 256 * 256
    for prob, prec, nrhs in [(W.gravity_1024(), "fp32", 1), (W.magnetic_48x56(), "fp64", 3)]:
        h = B.bttb_plan_create(prob, prec)
        sb, wb, _, _ = B.bttb_plan_query(h, nrhs)
        esz = 4 if prec == "fp32" else 8
        nx, ny, nz = W.dims(prob)
        want = up(sb) + up(wb) + up(nrhs * nx * ny * nz * esz) + up(nrhs * prob["sx"] * prob["sy"] * esz)
        need, avail = B.bttb_plan_memory_check(h, nrhs, want)
        assert (need, avail) == (want, want)
        with pytest.raises(B.BttbError) as e:
            B.bttb_plan_memory_check(h, nrhs, want - 1)
        assert e.value.status == 7 and "need" in str(e.value)
        n, a = ctypes.c_size_t(), ctypes.c_size_t()
        st = lib.bttb_plan_memory_check(ctypes.c_void_p(h), nrhs, want - 1, ctypes.byref(n), ctypes.byref(a))
        assert st == 7 and (n.value, a.value) == (want, want - 1)
        assert lib.bttb_plan_memory_check(ctypes.c_void_p(h), 0, want, None, None) == 1
        B.bttb_plan_destroy(h)
    assert _lib.load().bttb_plan_memory_check(None, 1, 1, None, None) == 2
    # the 1024 x 1024 x 128 FP32 volume with its spectra and workspace needs
    # about 2.03 GiB
    h = B.bttb_plan_create(W.gravity_1024(), "fp32")
    B.bttb_plan_memory_check(h, 1, 3 << 30)
    with pytest.raises(B.BttbError):
        B.bttb_plan_memory_check(h, 1, 2 << 30)
    B.bttb_plan_destroy(h)


def test_spectrum_form_choice(lib):
    import paper_1912_06976_amd as B
    cases = [
        (W.small_gravity(), "auto", "real_even"),
        (W.magnetic_48x56(), "auto", "complex"),
        (W.problem(W.PROBE, 3, 1, 1, dx=1.0, dy=1.0, dz=1.0), "auto", "complex"),
        # equal paddings: 2 (s - 1 + p) + 1 = s + n - 1 always fits
        (W.table1_problem(3, W.GRAVITY, True), "auto", "real_even"),
        # s + n - 1 = 15, but 2 (5 - 1 + 6) + 1 = 21 > 16: asked for N = 16
        (W.problem(W.GRAVITY, 5, 5, 2, 6, 0, 0, 0, dx=10.0, dy=10.0, dz=5.0, nx_fft=16), "auto", "complex"),
        # the same with room: N = 32, asked for or chosen by the plan
        (W.problem(W.GRAVITY, 5, 5, 2, 6, 0, 0, 0, dx=10.0, dy=10.0, dz=5.0, nx_fft=32), "auto", "real_even"),
        (W.problem(W.GRAVITY, 5, 5, 2, 6, 0, 0, 0, dx=10.0, dy=10.0, dz=5.0), "auto", "real_even"),
        (W.small_gravity(), "complex", "complex"),
    ]
    for pr, req, got in cases:
        h = B.bttb_plan_create(dict(pr, spectrum_form=req), "fp32")
        assert B.bttb_plan_spectrum_form(h) == got, (pr, req)
        B.bttb_plan_destroy(h)
    # the default length of an automatic-form gravity plan admits the real
    # even form; the complex form and the magnetic kernel take the smallest
    pr = W.problem(W.GRAVITY, 5, 5, 2, 6, 0, 0, 0, dx=10.0, dy=10.0, dz=5.0)
    for req, n in (("auto", 32), ("complex", 16)):
        h = B.bttb_plan_create(dict(pr, spectrum_form=req), "fp32")
        assert B.bttb_plan_query(h, 1)[2] == n, req
        B.bttb_plan_destroy(h)
    h = B.bttb_plan_create(dict(pr, kind=W.MAGNETIC, incl=60.0, decl=10.0), "fp32")
    assert B.bttb_plan_query(h, 1)[2] == 16
    B.bttb_plan_destroy(h)
    # (an explicit length that cannot hold the centred generator)
    for pr in (W.magnetic_48x56(), W.problem(W.GRAVITY, 5, 5, 2, 6, 0, 0, 0, dx=10.0, dy=10.0, dz=5.0, nx_fft=16),
               W.problem(W.TABLE, 5, 5, 2, 6, 0, 0, 0, nx_fft=16)):
        st, h, msg = _create(dict(pr, spectrum_form="real_even"))
        assert st == 3 and h.value is None and "REAL_EVEN" in msg
    # a user table is complex unless declared even
    for req, got in (("auto", "complex"), ("real_even", "real_even")):
        h = B.bttb_plan_create(dict(W.problem(W.TABLE, 13, 11, 5, 0, 3, 4, 1), spectrum_form=req), "fp32")
        assert B.bttb_plan_spectrum_form(h) == got
        B.bttb_plan_destroy(h)
    assert lib.bttb_plan_spectrum_form(None, None) == 2


def test_table_generation_argument_checks(lib):
    # fake (never dereferenced) device pointers: the checks fail first
    import paper_1912_06976_amd as B
    h = B.bttb_plan_create(W.problem(W.TABLE, 13, 11, 5, 0, 3, 4, 1), "fp64")
    g = B.bttb_plan_create(W.small_gravity(), "fp64")
    _, wb, _, _ = B.bttb_plan_query(h, 1)
    p = ctypes.c_void_p(1 << 20)
    assert lib.bttb_kernel_generate_table(ctypes.c_void_p(h), None, p, p, wb, None) == 2
    assert lib.bttb_kernel_generate_table(ctypes.c_void_p(g), p, p, p, wb, None) == 1
    assert lib.bttb_kernel_generate(ctypes.c_void_p(h), p, p, wb, None) == 1
    assert lib.bttb_kernel_generate_table(ctypes.c_void_p(h), p, p, p, wb - 1, None) == 4
    host = (ctypes.c_double * 4)()
    assert lib.bttb_debug_generator(ctypes.c_void_p(h), 0, host, p, 1 << 30, None) == 1
    B.bttb_plan_destroy(h)
    B.bttb_plan_destroy(g)


def test_workspace_too_small_is_rejected_before_launch(lib):
    # fake (never dereferenced) device pointers: the size check fails first
    import paper_1912_06976_amd as B
    h = B.bttb_plan_create(W.small_gravity(), "fp64")
    _, wb, _, _ = B.bttb_plan_query(h, 2)
    p = ctypes.c_void_p(1 << 20)
    assert lib.bttb_forward(ctypes.c_void_p(h), p, p, p, 2, p, wb - 1, None) == 4
    assert lib.bttb_transpose(ctypes.c_void_p(h), p, p, p, 2, p, wb - 1, None) == 4
    assert lib.bttb_forward(ctypes.c_void_p(h), p, p, p, 0, p, wb, None) == 1
    assert lib.bttb_kernel_generate(ctypes.c_void_p(h), ctypes.c_void_p(3), p, wb, None) == 1  # misaligned
    B.bttb_plan_destroy(h)


def test_overlapping_buffers_are_rejected(lib):
    # fake (never dereferenced) device pointers: the overlap check fails
    # before anything is enqueued
    import paper_1912_06976_amd as B
    h = B.bttb_plan_create(W.small_gravity(), "fp64")
    sb, wb, _, _ = B.bttb_plan_query(h, 1)
    assert sb < (1 << 28) and wb < (1 << 28)
    base = 1 << 32
    spec, ws, far = base, base + (1 << 28), base + (1 << 29)
    P = ctypes.c_void_p
    # input inside the workspace
    assert lib.bttb_forward(P(h), P(spec), P(ws + 256), P(far), 1, P(ws), wb, None) == 1
    # output inside the workspace
    assert lib.bttb_transpose(P(h), P(spec), P(far), P(ws + 512), 1, P(ws), wb, None) == 1
    # output over the spectra
    assert lib.bttb_transpose(P(h), P(spec), P(far), P(spec + 256), 1, P(ws), wb, None) == 1
    assert "overlap" in lib.bttb_last_error().decode()
    B.bttb_plan_destroy(h)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1912_06976_amd import _lib
    monkeypatch.setattr(_lib, "_handle", None)
    with pytest.raises(RuntimeError):
        _lib.load(str(tmp_path / "missing.so"))


def test_autotune_query_size(lib):
    from paper_1912_06976_amd.plan import make_desc
    import paper_1912_06976_amd as B
    d, keep = make_desc(W.gravity_1024(), "fp32")
    sz = ctypes.c_size_t()
    assert lib.bttb_autotune_query(ctypes.byref(d), 1, ctypes.byref(sz)) == 0
    h = B.bttb_plan_create(W.gravity_1024(), "fp32")
    sb, wb, _, _ = B.bttb_plan_query(h, 1)
    B.bttb_plan_destroy(h)
    vec = 2 * (1024 * 1024 * 128 + 1000 * 1000) * 4
    assert sb + wb + vec <= sz.value <= sb + wb + vec + 8 * 256
    assert lib.bttb_autotune_query(ctypes.byref(d), 0, ctypes.byref(sz)) == 1


def test_noalloc_forward_argument_checks(lib):
    # fake (never dereferenced) device pointers: every check here fails
    # before the library touches the device
    import paper_1912_06976_amd as B
    from paper_1912_06976_amd import _lib
    P = ctypes.c_void_p
    p = P(1 << 20)
    assert lib.bttb_forward_noalloc(None, p, p, p, 1, None) == 2
    h = B.bttb_plan_create(W.small_gravity(), "fp32")
    assert lib.bttb_forward_noalloc(P(h), p, p, p, 0, None) == 1
    B.bttb_plan_destroy(h)
    # a workspace above the scratch array's size is refused, with the sizes
    h = B.bttb_plan_create(W.gravity_1024(), "fp32")
    assert B.bttb_plan_query(h, 1)[1] > _lib.NOALLOC_SCRATCH_BYTES
    assert lib.bttb_forward_noalloc(P(h), p, p, p, 1, None) == 3
    msg = lib.bttb_last_error().decode()
    assert "bttb_forward_noalloc" in msg and str(_lib.NOALLOC_SCRATCH_BYTES) in msg
    B.bttb_plan_destroy(h)


def test_noalloc_scratch_size_matches_header():
    txt = open(os.path.join(ROOT, "include", "bttb.h")).read()
    from paper_1912_06976_amd import _lib
    m = re.search(r"#define BTTB_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.NOALLOC_SCRATCH_BYTES


def test_hessian_descriptor_checks(lib):
    import paper_1912_06976_amd as B
    base = W.problem(W.HESSIAN, 12, 10, 3, 1, 2, 0, 1, dx=50.0, dy=50.0, dz=25.0, hessian=(0, 0, 1, 0, 0, 0))
    st, _, msg = _create(dict(base, hessian=(0, 0, float("nan"), 0, 0, 0)))
    assert st == 1 and "hessian" in msg
    # off-diagonal weights make the kernel odd in an offset: no real even form
    st, _, msg = _create(dict(base, hessian=(0, 0, 1, 0, 0.5, 0), spectrum_form="real_even"))
    assert st == 3 and "REAL_EVEN" in msg
    for w, form in (((0, 0, 1, 0, 0, 0), "real_even"), ((1, -1, 0, 0, 0, 0), "real_even"),
                    ((0, 0, 1, 0.2, 0, 0), "complex")):
        h = B.bttb_plan_create(dict(base, hessian=w), "fp32")
        assert B.bttb_plan_spectrum_form(h) == form, w
        B.bttb_plan_destroy(h)


def test_grid_cap_hook_checks(lib):
    # host state only: no launch
    assert lib.bttb_debug_cap_grid(-1) == 1
    assert "max_blocks" in lib.bttb_last_error().decode()
    assert lib.bttb_debug_cap_grid(5) == 0
    assert lib.bttb_debug_cap_grid(0) == 0
