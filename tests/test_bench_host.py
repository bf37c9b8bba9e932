"""Host-side logic of bench.py (CPU): the one-GPU contract, the digest gate
on the committed HBM-traffic figure, and the workload configurations."""
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


def _profile(tmp_path, digest, value="123456789"):
    p = tmp_path / "traffic.md"
    p.write_text("# summary\n\n- gemm_source_sha256_16: `%s`\n- hbm_bytes_per_launch: `%s`\n" % (digest, value))
    return str(p)


def test_traffic_read_while_the_gemm_source_matches(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _profile(tmp_path, bench.gemm_source_digest()))
    assert bench.measured_traffic() == 123456789.0


def test_traffic_null_once_the_gemm_source_changed(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _profile(tmp_path, "0000000000000000"))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _profile(tmp_path, bench.gemm_source_digest(), "n/a"))
    assert bench.measured_traffic() is None


def test_workload_configs():
    a, b, eps, cfg = bench.workload("tiny")
    assert (a.nbr, a.nbc, b.nbc) == (100, 100, 100) and eps == 0.0
    assert cfg["workload"] == "tiny_100x100_blocks_5"
    with pytest.raises(SystemExit):
        bench.workload("no_such_workload")
