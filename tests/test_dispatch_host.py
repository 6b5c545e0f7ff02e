"""The class-grid dispatch tables, checked on the host (no device): the
geometry sources are compiled with g++ together with
tests/host/dispatch_table_check.cpp, which builds grids, a two-hop pattern
and a two-grid pair and checks every table: each member tile once, slot
8 i + x the i-th tile of XCD x, contiguous class-order ranges of equal work
run largest first, empty slots only at the ends; and the convolution chunks,
which cover every tile once and reach the workgroups largest first."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1504_04653_amd", "csrc")


def test_dispatch_tables(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "dispatch_table_check")
    res = subprocess.run(["g++", "-std=c++17", "-O1", "-ffp-contract=off", "-o", exe,
                          os.path.join(ROOT, "tests", "host", "dispatch_table_check.cpp"),
                          os.path.join(CSRC, "geometry.cpp")], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, (res.stdout + res.stderr)[-3000:]
    assert "dispatch_table_check OK" in res.stdout
