"""Host-side logic of bench.py (no GPU): the HBM byte model of the kernels,
the checks that tie the committed counter summary to the kernel source and
variant it was taken on, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_block_product_bytes_at_128x128x32():
    # packed spectral table: (Nx+1)(Ny+1) points x 2Nz(2Nz+1) complex128
    # (Sect. 3.1 storage); spectra: R vectors x 3Nz planes x 2Nx x 2Ny,
    # read once and written once
    table = 129 * 129 * (64 * 65) * 16
    spectra = 2 * 96 * 256 * 256 * 16
    assert table == 1_107_624_960 and spectra == 201_326_592
    assert bench.stage_bytes(128, 128, 32, 2, 16)["block_product"] == table + 2 * spectra
    # the three-step model adds 78 N c per right-hand side to the table
    assert bench.m3_bytes(128, 128, 32, 2, 16) == table + 2 * 78 * 128 * 128 * 32 * 16


def test_counter_summary_is_tied_to_source_and_variant(tmp_path, monkeypatch):
    import hashlib
    src = tmp_path / "kernels_block.hip"
    src.write_bytes(b"// a kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summary = tmp_path / "counters.md"
    summary.write_text("# counters\n\n"
                       f"- kernel_source_sha256: `{sha}`\n"
                       "- block_buffers: `2`\n"
                       "- hbm_bytes_per_launch: `1.543681e+09`\n")
    monkeypatch.setattr(bench, "BLOCK_SOURCE", str(src))
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(summary))
    assert bench.read_traffic(2) == 1.543681e9
    assert bench.read_traffic(1) is None            # taken on variant 2 only
    src.write_bytes(b"// a kernel source\n// edited\n")
    assert bench.read_traffic(2) is None            # kernel changed since
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(tmp_path / "absent.md"))
    assert bench.read_traffic(2) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
