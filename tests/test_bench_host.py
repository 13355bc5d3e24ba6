"""Host-side parts of bench.py (CPU): the one-GPU rule and the byte / flop
models of the roofline, checked against hand-counted values for the bench
volume."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_of_the_bench_volume():
    import bench
    import workloads as W
    pr = W.gravity_1024()
    nx, ny, nz = W.dims(pr)
    assert (nx, ny, nz) == (1024, 1024, 128)
    # real even spectra: nz (Nx/2 + 1) (Ny/2 + 1) floats; complex: nz (Nx/2) Ny complex
    assert bench.spectra_bytes(pr, 2048, 2048, 4, "real_even") == 128 * 1025 * 1025 * 4
    assert bench.spectra_bytes(pr, 2048, 2048, 4, "complex") == 128 * 1024 * 2048 * 8
    # one G m + G^T r: spectra twice, m and G^T r, r and d
    pb = bench.pair_bytes(pr, 2048, 2048, 4, "real_even")
    assert pb == 2 * 128 * 1025 * 1025 * 4 + 2 * 1024 * 1024 * 128 * 4 + 2 * 1000 * 1000 * 4
    kb = bench.kernel_bytes(pr, 2048, 2048, 4, "real_even")
    # the forward MAC reads X (nz half-spectrum panels of 1024 columns by ny
    # rows, complex) and the spectra, and writes Y (1024 columns by sy rows)
    x = 128 * 1024 * 1024 * 8
    assert kb["fwd_cols_fft_mac"] == x + 128 * 1025 * 1025 * 4 + 1024 * 1000 * 8
    assert kb["fwd_rows_r2c"] == 1024 * 1024 * 128 * 4 + x
    # the dominant kernel's flops: 5 N log2 N per column FFT (nz + 1 per
    # column) plus the real-by-complex products
    kf = bench.kernel_flops(pr, 2048, 2048, "real_even")
    assert kf["fwd_cols_fft_mac"] > 1024 * 128 * 5 * 2048 * 11


def test_kernel_source_hash_covers_every_kernel_source():
    import bench
    src = os.path.join(ROOT, "paper_1912_06976_amd", "csrc")
    kernel_files = {f for f in os.listdir(src) if f.endswith((".hip", ".h"))} - {"bttb_host.hip", "bttb_cgls.hip"}
    assert kernel_files == set(bench.KERNEL_SOURCES)


def test_kernel_source_hash_ignores_comments(tmp_path, monkeypatch):
    import bench
    h0 = bench.kernel_source_hash()
    src = os.path.join(ROOT, "paper_1912_06976_amd", "csrc")
    copy = tmp_path / "paper_1912_06976_amd" / "csrc"
    copy.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        text = open(os.path.join(src, f)).read()
        if f == "fft_core.h":
            text = "// an added comment line\n" + text.replace("\n", "  \n", 3)
        (copy / f).write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h0
    (copy / "kern_common.h").write_text((copy / "kern_common.h").read_text() + "\nint changed_code;\n")
    assert bench.kernel_source_hash() != h0


def test_traffic_needs_the_counters_kernel_config(tmp_path, monkeypatch):
    """Counter bytes are per launch of one kernel configuration: a run with
    layer chunks (other launches) gets no traffic figure."""
    import json
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    info = {"source_sha256": bench.kernel_source_hash(), "kernel_config": bench.DEFAULT_KERNEL_CONFIG,
            "kernels": {"tr_cols_fft_mac": {"read_bytes": 5, "write_bytes": 7}}}
    (prof / "hbm_counters_gravity_1024_fp32.md").write_text("<!-- traffic-json: %s -->\n" % json.dumps(info))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: info["source_sha256"])
    assert bench.counter_traffic("tr_cols_fft_mac", bench.effective_kernel_config({})) == 12
    assert bench.counter_traffic("tr_cols_fft_mac", bench.effective_kernel_config({"layer_chunk": 32})) is None
    assert bench.counter_traffic("tr_cols_fft_mac", bench.effective_kernel_config({"row_tile": 2})) is None
    assert bench.counter_traffic("tr_cols_fft_mac", dict(bench.DEFAULT_KERNEL_CONFIG)) == 12
