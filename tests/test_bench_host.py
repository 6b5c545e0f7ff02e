"""bench.py on the host: the one-GPU refusal, argument defaults, and the
traffic lookup that keys counter rows by the kernel source hash."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused_with_a_message(n):
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_default_arguments():
    old = sys.argv
    try:
        sys.argv = ["bench.py"]
        a = bench.parse()
        assert (a.gpus, a.config, a.op) == (1, "lmax3000", "btnb")
        assert a.modes.split(",")[0] == "bf16x6"
        sys.argv = ["bench.py", "--config", "batch32"]
        assert bench.parse().modes.split(",")[0] == "bf16x6"
    finally:
        sys.argv = old


def test_traffic_rows_count_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    h = bench.kernels_hash()
    (prof / "pmc_traffic.md").write_text(
        f"| bf16x6 | lmax3000 | {h} | 1.0e+08 | 2.0e+09 |\n"
        f"| fp64 | lmax3000 | 0000000000000000 | 5.0e+08 | 6.0e+09 |\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernels_hash", lambda: h)
    assert bench.recorded_traffic("bf16x6", "lmax3000") == pytest.approx(2.1e9)
    assert bench.recorded_traffic("fp64", "lmax3000") is None        # taken on another source
    assert bench.recorded_traffic("bf16x6", "batch32") is None      # no row
