"""bench.py on the host: the one-GPU refusal, argument defaults, and the
traffic lookup that keys counter rows by the kernel source hash."""
import os
import subprocess
import sys

import numpy as np
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
        assert a.modes.split(",") == ["fp64", "bf16x6", "fp32", "bf16x3"]   # value is plain FP64
        assert bench.HEADLINE == "fp64"
        sys.argv = ["bench.py", "--config", "batch32"]
        assert bench.parse().modes.split(",")[0] == "fp32"                 # FP32 MFMA leads the batch
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
    monkeypatch.setattr(bench, "kernels_hash", lambda source="kernels.hip": h)
    assert bench.recorded_traffic("bf16x6", "lmax3000") == pytest.approx(2.1e9)
    assert bench.recorded_traffic("fp64", "lmax3000") is None        # taken on another source
    assert bench.recorded_traffic("bf16x6", "batch32") is None      # no row


def test_sampled_rows_start_with_the_special_bands():
    """Polar, equatorial and ratio-transition bands first (their first tiles),
    then distinct random tiles."""
    tiles = [18, 18, 27, 27, 54, 54, 72, 72]      # storage order N0, S0, N1, S1, ...
    t0 = [0, 18, 36, 63, 90, 144, 198, 270]
    rows = bench.sampled_rows(tiles, 20, seed=1)
    assert rows[:4] == [t0[0], t0[1], t0[6], t0[7]]
    assert rows[4:8] == [t0[2], t0[3], t0[4], t0[5]]      # every other band borders a change of T
    assert len(rows) == 8 + 20
    assert len(rows) == len(set(rows)) and all(0 <= r < sum(tiles) for r in rows)
    assert len(bench.sampled_rows([1, 1], 50, seed=2)) == 2       # no more rows than tiles


def test_cpu_baseline_reports_each_modes_error_against_the_oracle():
    """The cpu_baseline leg times the oracle on the sampled rows and compares
    every mode's outputs of those rows with it: an exact copy gives gate 0, an
    output off by 1e-7 of the row maximum in one element gives 1e-7."""
    import paper_1504_04653_amd as sp
    from oracle import grid as G
    from oracle import operators as O
    from workloads import synth as S
    cfg = S.CONFIGS["lmax64"]
    g = sp.Grid(cfg.lmax, cfg.k)
    rows = bench.sampled_rows(g.bands()[0], 4, seed=3)
    rp, col = g.blocks()
    idx, pairs = bench.row_blocks(rp, col, rows)
    og = G.make_grid(cfg.lmax, cfg.k)
    ring, _, _, phi = og.pixel_coords()
    ninv = S.ninv_for(cfg, og.theta[ring], phi)
    b_l, R = S.gaussian_beam(cfg.lmax, og.npix, cfg.fwhm_pix)
    C = O.sample_BtNB(og, b_l, ninv, R, pairs)
    D = O.sample_D(og, S.prior(cfg.lmax), None, pairs)
    off = C.copy()
    mj = np.abs(C[0:len([p for p in pairs if p[0] == pairs[0][0]])]).max()
    off[0, 3, 5] += 1e-7 * mj
    sampled = {"rows": rows, "pairs": pairs,
               "modes": {"fp64": {"C": C, "D": D}, "bf16x6": {"C": off, "D": None}}}
    base, gates = bench.cpu_baseline(cfg, g, 0.2, 0.0, sampled)
    assert base["kind"] == "oracle" and base["value"] > 0 and base["layout_matches_oracle"]
    assert {"nproc", "cpu_model"} <= set(base["host"])
    assert gates["fp64"]["C"]["gate"] == 0.0 and gates["fp64"]["D"]["gate"] == 0.0
    assert gates["bf16x6"]["C"]["gate"] == pytest.approx(1e-7, rel=1e-6)
    assert "D" not in gates["bf16x6"]
