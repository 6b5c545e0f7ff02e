"""GPU parity of the two-grid operator B-hat = Y_2 B Y_1^T (Eqs. 13, 16) and
B-hat^T N_2^-1 B-hat (Eq. 15) through the C ABI, against the FP64 oracle
(oracle.twogrid): every block on small grid pairs in every precision mode,
sampled block-rows at lmax 1500 with Y_2 at lmax 3000 (the paper's "twice the
band limit of Y_1"), and the limit Y_2 = Y_1, where every output must be
bitwise that of the one-grid calls."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1504_04653_amd as sp
from oracle import grid as G
from oracle import operators as O
from oracle import twogrid as X
from workloads import synth as S

from _parity import error_report, sample_rows

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


def run_cross(x, kb, n2, prec):
    out = torch.full((x.out_len,), float("nan"), dtype=torch.float64, device="cuda")
    sp.sample_BtNB_cross(x, kb, n2, out, prec)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("lmax", [16, 64, 256])
def test_equal_grids_are_bitwise_the_one_grid_calls(lmax):
    g = sp.Grid(lmax, 8)
    x = sp.Cross(g, g)
    rng = np.random.default_rng(50 + lmax)
    ninv = rng.uniform(0.5, 2.0, g.npix)
    ninv[rng.random(g.npix) < 0.1] = 0.0
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    kb = sp.Kernel(g, b_l, R)
    kx = sp.CrossKernel(x, b_l, R)
    n_dev = dev(ninv)
    for prec in MODES:
        ref = torch.empty(g.out_len, dtype=torch.float64, device="cuda")
        sp.sample_BtNB(g, kb, n_dev, ref, prec)
        got = run_cross(x, kx, n_dev, prec)
        assert torch.equal(got, ref), f"lmax {lmax} {prec}: two-grid call with Y_2 = Y_1 differs from sample_BtNB"
    # B-hat blocks: entries (I, J >= I) are the stored blocks sample_D returns for the beam kernel
    B = torch.empty(x.b_len, dtype=torch.float64, device="cuda")
    sp.sample_B_cross(x, kx, B)
    Dst = torch.empty(g.out_len, dtype=torch.float64, device="cuda")
    sp.sample_D(g, kb, Dst)
    torch.cuda.synchronize()
    _, rp, col, _ = x.neighbours()
    keep = [e for I in range(g.ntiles) for e in range(rp[I], rp[I + 1]) if col[e] >= I]
    assert torch.equal(B.view(-1, 64, 64)[torch.as_tensor(keep, device="cuda")], Dst.view(-1, 64, 64))
    say(f"[twogrid {lmax}] Y_2 = Y_1: B-hat blocks and B^T N^-1 B in every mode bitwise equal to the one-grid calls")


# (32, 128) and (48, 128): Y_2 coarser than half of Y_1's resolution, where
# some stored blocks (J, K) have no tile of Y_2 neighbouring both (an empty sum
# in Eq. 15: zero blocks, a class without terms)
PAIRS = [(128, 64), (100, 64), (64, 128), (512, 256), (32, 128), (48, 128)]


@pytest.mark.parametrize("l2,l1", PAIRS)
def test_small_pairs_every_block_against_oracle(l2, l1):
    og2, og1 = G.make_grid(l2, 8), G.make_grid(l1, 8)
    g2, g1 = sp.Grid(l2, 8), sp.Grid(l1, 8)
    x = sp.Cross(g2, g1)
    rng = np.random.default_rng(7 * l2 + l1)
    ninv2 = rng.uniform(0.5, 2.0, g2.npix)
    ninv2[rng.random(g2.npix) < 0.1] = 0.0
    b_l, R = S.gaussian_beam(l1, g1.npix, 3.0)
    kx = sp.CrossKernel(x, b_l, R)
    say(f"[twogrid {l2}/{l1}] npix2={g2.npix} npix1={g1.npix} blocks={x.nblocks} B-hat blocks={x.nadjacency} "
        f"terms={x.nterms} (max {x.max_terms}) unique={x.nunique}")
    # B-hat blocks (first 3000 in relation order)
    B = torch.empty(x.b_len, dtype=torch.float64, device="cuda")
    sp.sample_B_cross(x, kx, B)
    torch.cuda.synchronize()
    op = X.CrossOperator(og2, og1, b_l, R)
    _, rp, col, _ = x.neighbours()
    ent = [(I, int(col[e]), e) for I in range(g2.ntiles) for e in range(rp[I], rp[I + 1])][:3000]
    Bref = np.stack([op.block(I, J) for I, J, _ in ent])
    Bgot = B.view(-1, 64, 64)[torch.as_tensor([e for _, _, e in ent], device="cuda")].cpu().numpy()
    errB = np.abs(Bgot - Bref).max() / np.abs(Bref).max()
    say(f"[twogrid {l2}/{l1}] B-hat blocks: max err / peak {errB:.3e}")
    assert errB <= 1e-12
    pairs = O.stored_block_list(og1)
    rows = [J for J, _ in pairs]
    Cref = X.sample_BtNB_cross(og2, og1, b_l, ninv2, R, pairs)
    n_dev = dev(ninv2)
    for prec in MODES:
        C = run_cross(x, kx, n_dev, prec).view(-1, 64, 64).cpu().numpy()
        rep = error_report(C, Cref, rows)
        say(f"[twogrid {l2}/{l1}] BtNB {prec}: {rep}")
        assert rep["gate"] <= GATE[prec]


def test_full_size_lmax1500_with_auxiliary_lmax3000_sampled():
    cfg = S.CONFIGS["lmax1500"]
    og1, og2 = G.make_grid(1500, 8), G.make_grid(3000, 8)
    g1, g2 = sp.Grid(1500, 8), sp.Grid(3000, 8)
    x = sp.Cross(g2, g1)
    th2, ph2 = g2.pixel_theta_phi()
    ninv2 = S.ninv_for(cfg, th2, ph2)
    b_l, R = S.gaussian_beam(1500, g1.npix, cfg.fwhm_pix)
    kx = sp.CrossKernel(x, b_l, R)
    rows = sample_rows(og1, 8, seed=cfg.seed + 11)
    brp, bcol = g1.blocks()
    idx, pairs = [], []
    for J in rows:
        ks = [K for K in og1.tile_neighbours(J) if K >= J]
        assert bcol[brp[J]:brp[J + 1]].tolist() == ks
        for n, K in zip(range(brp[J], brp[J + 1]), ks):
            idx.append(n)
            pairs.append((J, K))
    say(f"[twogrid 3000/1500] npix2={g2.npix} blocks={x.nblocks} terms={x.nterms} (max {x.max_terms}) "
        f"unique={x.nunique}; sampled rows={len(rows)} blocks={len(idx)}")
    op = X.CrossOperator(og2, og1, b_l, R)
    Cref = np.stack([X.btnb_cross_block(op, ninv2, J, K) for J, K in pairs])
    idx_t = torch.as_tensor(idx, device="cuda")
    n_dev = dev(ninv2)
    for prec in MODES:
        C = run_cross(x, kx, n_dev, prec)
        assert not bool(torch.isnan(C).any()), f"{prec}: a block was not written"
        rep = error_report(C.view(-1, 64, 64)[idx_t].cpu().numpy(), Cref, [J for J, _ in pairs])
        say(f"[twogrid 3000/1500] BtNB {prec}: {rep}")
        assert rep["gate"] <= GATE[prec]
        del C
        torch.cuda.empty_cache()


def test_two_grid_errors():
    g1, g2 = sp.Grid(64, 8), sp.Grid(128, 8)
    x = sp.Cross(g2, g1)
    b_l, R = S.gaussian_beam(64, g1.npix, 3.0)
    kx = sp.CrossKernel(x, b_l, R)
    kb = sp.Kernel(g1, b_l, R)
    n2 = torch.ones(g2.npix, dtype=torch.float64, device="cuda")
    out = torch.zeros(x.out_len, dtype=torch.float64, device="cuda")
    for bad in (lambda: sp.sample_BtNB_cross(x, kx, n2[:-1], out, "fp64"),
                lambda: sp.sample_BtNB_cross(x, kx, n2, out[:-1], "fp64"),
                lambda: sp.sample_B_cross(x, kx, out[:5])):
        with pytest.raises(sp.SympixError) as ei:
            bad()
        assert ei.value.code == "ESIZE"
    with pytest.raises(sp.SympixError) as ei:                   # a one-grid kernel
        sp.sample_BtNB_cross(x, kb, n2, out, "fp64")
    assert ei.value.code == "EINVAL"
    with pytest.raises(sp.SympixError) as ei:                   # a two-grid kernel in a one-grid call
        sp.sample_BtNB(g1, kx, torch.ones(g1.npix, dtype=torch.float64, device="cuda"), out, "fp64")
    assert ei.value.code == "EINVAL"
    x2 = sp.Cross(g2, g1)
    with pytest.raises(sp.SympixError) as ei:                   # kernel of another pair
        sp.sample_BtNB_cross(x2, kx, n2, out, "fp64")
    assert ei.value.code == "EINVAL"
    with pytest.raises(sp.SympixError) as ei:
        sp.sample_BtNB_cross(x, kx, n2, out, 9)
    assert ei.value.code == "EINVAL"
    assert int(torch.count_nonzero(out)) == 0, "a failed call wrote output"
