"""GPU parity of the combined call sample_D_BtNB (both local operators of
Eq. 16 in one call; one launch in the split-BF16 modes).

Its two outputs must be bitwise equal to the separate calls sample_D and
sample_BtNB in the same mode, which the parity tests hold to the oracle; the
fused outputs are also checked against the oracle directly on sampled
block-rows of the lmax 3000 workload (the launch configuration bench.py
times).  Grids run from one band per hemisphere (lmax 1) to lmax 3000, so
tiles of 16, 32 and 64 member rows, classes of one to sixteen terms, and the
D-hat chunks copied after a tile's last step are all exercised.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1504_04653_amd as sp
from oracle import grid as G
from oracle import operators as O
from workloads import synth as S

from _parity import block_index, config_inputs, error_report, sample_rows

pytestmark = pytest.mark.gpu

GATE = {"fp64": 1e-10, "fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 2.0 ** -15}
MODES = ("fp64", "fp32", "bf16x6", "bf16x3")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def nan_buffer(n):
    return torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")


def separate(g, kd, kb, n_dev, prec):
    D = nan_buffer(g.out_len)
    C = nan_buffer(g.out_len)
    sp.sample_D(g, kd, D)
    sp.sample_BtNB(g, kb, n_dev, C, prec)
    torch.cuda.synchronize()
    return D, C


def fused(g, kd, kb, n_dev, prec):
    D = nan_buffer(g.out_len)
    C = nan_buffer(g.out_len)
    sp.sample_D_BtNB(g, kd, kb, n_dev, D, C, prec)
    torch.cuda.synchronize()
    return D, C


@pytest.mark.parametrize("lmax", [1, 7, 16, 40, 64, 256])
def test_fused_equals_separate_calls(lmax):
    g = sp.Grid(lmax, 8)
    rng = np.random.default_rng(3000 + lmax)
    ninv = rng.uniform(0.5, 2.0, g.npix)
    ninv[rng.random(g.npix) < 0.1] = 0.0
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    kb = sp.Kernel(g, b_l, R)
    kd = sp.Kernel(g, S.prior(lmax), 0.0)
    n_dev = dev(ninv)
    say(f"[fused {lmax}] npix={g.npix} nblocks={g.nblocks} nterms={g.nterms}")
    for prec in MODES:
        D0, C0 = separate(g, kd, kb, n_dev, prec)
        D1, C1 = fused(g, kd, kb, n_dev, prec)
        assert torch.equal(D1, D0), f"lmax {lmax} {prec}: D-hat differs from sample_D"
        assert torch.equal(C1, C0), f"lmax {lmax} {prec}: B^T N^-1 B differs from sample_BtNB"
        say(f"[fused {lmax}] {prec}: both outputs bitwise equal to the separate calls")


def test_fused_full_size_against_oracle_and_separate_calls():
    cfg = S.CONFIGS["lmax3000"]
    og = G.make_grid(cfg.lmax, cfg.k)
    g = sp.Grid(cfg.lmax, cfg.k)
    ninv, b_l, R, d_l = config_inputs(cfg, og)
    kb = sp.Kernel(g, b_l, R)
    kd = sp.Kernel(g, d_l, 0.0)
    n_dev = dev(ninv)
    rows = sample_rows(og, 6, seed=cfg.seed + 1)
    brp, bcol = g.blocks()
    idx, pairs = block_index(og, brp, bcol, rows)
    jrow = [J for J, _ in pairs]
    idx_t = torch.as_tensor(idx, device="cuda")
    op = O.LocalOperator(og, b_l, R)
    Cref = np.stack([O.btnb_block(op, ninv, J, K) for J, K in pairs])
    Dref = O.sample_D(og, d_l, None, pairs)
    say(f"[fused lmax3000] npix={g.npix} nblocks={g.nblocks} sampled rows={len(rows)} blocks={len(idx)}")
    for prec in MODES:
        D1, C1 = fused(g, kd, kb, n_dev, prec)
        rep_c = error_report(C1.view(-1, 64, 64)[idx_t].cpu().numpy(), Cref, jrow)
        rep_d = error_report(D1.view(-1, 64, 64)[idx_t].cpu().numpy(), Dref, jrow)
        say(f"[fused lmax3000] {prec}: C {rep_c}; D {rep_d}")
        assert rep_c["gate"] <= GATE[prec]
        assert rep_d["gate"] <= GATE["fp64"]
        assert not bool(torch.isnan(D1).any()), f"{prec}: a D-hat block was not written"
        assert not bool(torch.isnan(C1).any()), f"{prec}: a B^T N^-1 B block was not written"
        D0, C0 = separate(g, kd, kb, n_dev, prec)
        assert torch.equal(D1, D0), f"lmax3000 {prec}: D-hat differs from sample_D"
        assert torch.equal(C1, C0), f"lmax3000 {prec}: B^T N^-1 B differs from sample_BtNB"
        say(f"[fused lmax3000] {prec}: both outputs bitwise equal to the separate calls")
        del D0, C0, D1, C1
        torch.cuda.empty_cache()


def test_fused_argument_errors():
    g = sp.Grid(64, 8)
    b_l, R = S.gaussian_beam(64, g.npix, 3.0)
    kb = sp.Kernel(g, b_l, R)
    kd = sp.Kernel(g, S.prior(64), 0.0)
    n_dev = dev(np.ones(g.npix))
    D = torch.zeros(g.out_len, dtype=torch.float64, device="cuda")
    C = torch.zeros(g.out_len, dtype=torch.float64, device="cuda")
    with pytest.raises(sp.SympixError) as ei:
        sp.sample_D_BtNB(g, kd, kb, n_dev, C, C, "bf16x6")         # outputs overlap
    assert ei.value.code == "EINVAL"
    with pytest.raises(sp.SympixError) as ei:
        sp.sample_D_BtNB(g, kd, kb, n_dev, D[:-1], C, "bf16x6")
    assert ei.value.code == "ESIZE"
    other = sp.Grid(16, 8)
    k_other = sp.Kernel(other, S.prior(16), 0.0)
    with pytest.raises(sp.SympixError) as ei:
        sp.sample_D_BtNB(g, k_other, kb, n_dev, D, C, "bf16x6")    # D-hat kernel of another grid
    assert ei.value.code == "EINVAL"
    both = torch.zeros(2 * g.out_len + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(sp.SympixError) as ei:                       # misaligned D-hat output
        sp.sample_D_BtNB(g, kd, kb, n_dev, both[1:g.out_len + 1], C, "bf16x6")
    assert ei.value.code == "EINVAL"
    assert int(torch.count_nonzero(D)) == 0 and int(torch.count_nonzero(C)) == 0, "a failed call wrote output"
