"""Host-side logic of bench.py (CPU): the one-GPU contract, the digest gate
on the committed counter figures, and the workload configurations."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", ["2", "8"])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", n],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")   # no result line


def _profile(tmp_path, digest, value="123456789", name="k_gemm_f64_dft4000_traffic.md"):
    (tmp_path / name).write_text("# summary\n\n- source_sha256_16: `%s`\n- hbm_bytes_per_launch: `%s`\n"
                                 "- mfma_busy_frac: `0.25`\n" % (digest, value))
    return str(tmp_path)


def test_counters_read_while_the_kernel_source_matches(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", _profile(tmp_path, bench.source_digest("gemm_kernels.hip")))
    assert bench.profile_values("packed", "dft4000", "traffic")["hbm_bytes_per_launch"] == 123456789.0
    r = bench.roofline("packed", "dft4000", 1e12, 10.0, 1000)
    assert r["traffic"] == 123456789.0 and r["frac"] == round(100.0 / bench.FP64_MFMA_PEAK_TFLOPS, 4)
    assert r["mfma_busy"] is None   # no mfma summary in this folder
    # the tile kernel's summaries are keyed to its own source
    _profile(tmp_path, bench.source_digest("tile_gemm.hip"), name="k_tile_gemm_panel23_mfma.md")
    assert bench.roofline("tile", "panel23", 1e12, 10.0, 1000)["mfma_busy"] == 0.25


def test_counters_null_once_the_kernel_source_changed(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", _profile(tmp_path, "0000000000000000"))
    assert bench.profile_values("packed", "dft4000", "traffic") == {}
    assert bench.roofline("packed", "dft4000", 1e12, 10.0, 1000)["traffic"] is None
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path / "missing"))
    assert bench.profile_values("packed", "dft4000", "traffic") == {}
    monkeypatch.setattr(bench, "PROFILE_DIR",
                        _profile(tmp_path, bench.source_digest("gemm_kernels.hip"), "n/a"))
    assert "hbm_bytes_per_launch" not in bench.profile_values("packed", "dft4000", "traffic")
    # a summary of another kernel's source does not count for this one
    monkeypatch.setattr(bench, "PROFILE_DIR",
                        _profile(tmp_path, bench.source_digest("tile_gemm.hip")))
    assert bench.profile_values("packed", "dft4000", "traffic") == {}


def test_workload_configs():
    a, b, eps, cfg = bench.workload("tiny")
    assert (a.nbr, a.nbc, b.nbc) == (100, 100, 100) and eps == 0.0
    assert cfg["workload"] == "tiny_100x100_blocks_5"
    with pytest.raises(SystemExit):
        bench.workload("no_such_workload")
