"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Gates (max |GPU - oracle| / M_J, M_J the largest oracle value of block-row J):
FP64 1e-10; FP32 and BF16X6 1e-6.  BF16X3 (two-part split) is reported and
held to 2^-15: its products err by up to about 2^-16, and a sum may be half the
sum of its absolute products.  Every test prints the per-element error
distribution.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1504_04653_amd as sp
from oracle import grid as G
from oracle import kernel as OK
from oracle import operators as O
from workloads import synth as S

from _parity import block_index, config_inputs, error_report, gate, sample_rows, stored_pairs

pytestmark = pytest.mark.gpu

GATE = {"fp64": 1e-10, "fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 2.0 ** -15}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def run_D(g, kern):
    out = torch.empty(g.out_len, dtype=torch.float64, device="cuda")
    sp.sample_D(g, kern, out)
    torch.cuda.synchronize()
    return out.view(g.nblocks, 64, 64)


def run_BtNB(g, kern, ninv_dev, prec):
    out = torch.empty(g.out_len, dtype=torch.float64, device="cuda")
    sp.sample_BtNB(g, kern, ninv_dev, out, prec)
    torch.cuda.synchronize()
    return out.view(g.nblocks, 64, 64)


# --- C1: lmax 64, every block against the oracle ----------------------------

@pytest.fixture(scope="module")
def lmax64():
    cfg = S.CONFIGS["lmax64"]
    og = G.make_grid(cfg.lmax, cfg.k)
    g = sp.Grid(cfg.lmax, cfg.k)
    ninv, b_l, R, d_l = config_inputs(cfg, og)
    pairs = stored_pairs(og)
    rows = [J for J, _ in pairs]
    say(f"[lmax64] npix={g.npix} nblocks={g.nblocks} nterms={g.nterms} nunique={g.nunique}")
    return dict(og=og, g=g, ninv=ninv, b_l=b_l, R=R, d_l=d_l, pairs=pairs, rows=rows,
                kb=sp.Kernel(g, b_l, R), kd=sp.Kernel(g, d_l, 0.0))


def test_lmax64_kernel_table_interpolation(lmax64):
    """The table's 4-point interpolation against the oracle's direct sum at
    random y over the whole domain: <= 1e-12 of the kernel's peak."""
    g = lmax64["g"]
    rng = np.random.default_rng(1)
    for name, coef, R in (("beam", lmax64["b_l"], lmax64["R"]), ("prior", lmax64["d_l"], None)):
        kern = lmax64["kb"] if name == "beam" else lmax64["kd"]
        ydom = g.y_pattern_max if R is None else min(g.y_pattern_max, 2 * math.sin(R / 2) ** 2)
        y = np.concatenate([[0.0], rng.uniform(0, ydom, 4000), ydom * rng.uniform(0, 1e-4, 200)])
        out = torch.empty(y.size, dtype=torch.float64, device="cuda")
        kern.eval(dev(y), out)
        ref = OK.legendre_series_in_y(coef, y)
        peak = abs(OK.legendre_series_in_y(coef, np.array([0.0]))[0])
        err = np.abs(out.cpu().numpy() - ref).max() / peak
        say(f"[lmax64] table {name}: max err / peak = {err:.3e}")
        assert err <= 1e-12


@pytest.mark.parametrize("name", ["lmax512", "lmax1500", "lmax3000"])
def test_kernel_table_interpolation_full_size(name):
    """The 2^16-node table of the beam and of the prior d_l = (l+1)^2 (which
    oscillates fastest at high lmax) against the oracle's direct Legendre sum
    in y, at random y over the whole table domain and near y = 0: <= 1e-13 of
    the kernel's peak."""
    cfg = S.CONFIGS[name]
    g = sp.Grid(cfg.lmax, cfg.k)
    b_l, R = S.gaussian_beam(cfg.lmax, g.npix, cfg.fwhm_pix)
    rng = np.random.default_rng(cfg.seed + 5)
    for kname, coef, rad in (("beam", b_l, R), ("prior", S.prior(cfg.lmax), None)):
        kern = sp.Kernel(g, coef, 0.0 if rad is None else rad)
        ydom = g.y_pattern_max if rad is None else min(g.y_pattern_max, 2 * math.sin(rad / 2) ** 2)
        y = np.concatenate([[0.0], rng.uniform(0, ydom, 1500), ydom * rng.uniform(0, 1e-3, 100),
                            ydom * (1.0 - rng.uniform(0, 1e-3, 20))])
        out = torch.empty(y.size, dtype=torch.float64, device="cuda")
        kern.eval(dev(y), out)
        torch.cuda.synchronize()
        ref = OK.legendre_series_in_y(coef, y)
        peak = abs(OK.legendre_series_in_y(coef, np.array([0.0]))[0])
        err = np.abs(out.cpu().numpy() - ref).max() / peak
        say(f"[{name}] table {kname}: max err / peak = {err:.3e} over {y.size} points")
        assert err <= 1e-13
        del kern


def test_lmax64_D_and_B_blocks(lmax64):
    og, g, pairs, rows = lmax64["og"], lmax64["g"], lmax64["pairs"], lmax64["rows"]
    D = run_D(g, lmax64["kd"]).cpu().numpy()
    Dref = O.sample_D(og, lmax64["d_l"], None, pairs)
    rep = error_report(D, Dref, rows)
    say(f"[lmax64] D fp64: {rep}")
    assert rep["gate"] <= GATE["fp64"]
    B = run_D(g, lmax64["kb"]).cpu().numpy()
    Bref = O.sample_D(og, lmax64["b_l"], lmax64["R"], pairs)
    rep = error_report(B, Bref, rows)
    say(f"[lmax64] B fp64: {rep}")
    assert rep["gate"] <= GATE["fp64"]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3"])
def test_lmax64_btnb(lmax64, prec):
    og, g, pairs, rows = lmax64["og"], lmax64["g"], lmax64["pairs"], lmax64["rows"]
    if "Cref" not in lmax64:
        lmax64["Cref"] = O.sample_BtNB(og, lmax64["b_l"], lmax64["ninv"], lmax64["R"], pairs)
    C = run_BtNB(g, lmax64["kb"], dev(lmax64["ninv"]), prec).cpu().numpy()
    rep = error_report(C, lmax64["Cref"], rows)
    say(f"[lmax64] BtNB {prec}: {rep}")
    assert rep["gate"] <= GATE[prec]


def test_lmax64_fp64_is_bitwise_reproducible(lmax64):
    g = lmax64["g"]
    n = dev(lmax64["ninv"])
    a = run_BtNB(g, lmax64["kb"], n, "fp64").clone()
    b = run_BtNB(g, lmax64["kb"], n, "fp64")
    assert torch.equal(a, b)


def test_lmax64_delta_map_and_linearity(lmax64):
    """N^-1 = e_p gives rank-one blocks B(p, J_a) B(p, K_b); the result is linear
    in N^-1 (Eq. 15 closed forms, checked on the GPU output alone)."""
    g = lmax64["g"]
    Bblk = run_D(g, lmax64["kb"]).cpu().numpy()                 # local B-hat blocks
    brp, bcol = g.blocks()
    p = 5 * 64 + 17                                           # a pixel of tile 5
    w = np.zeros(g.npix)
    w[p] = 1.0
    C = run_BtNB(g, lmax64["kb"], dev(w), "fp64").cpu().numpy()
    rows = np.repeat(np.arange(g.ntiles), np.diff(brp))
    Bfull = {}
    for n, (J, K) in enumerate(zip(rows, bcol)):
        Bfull[(J, int(K))] = Bblk[n]
        Bfull[(int(K), J)] = Bblk[n].T
    I, a = divmod(p, 64)
    peak = max(np.abs(Bblk).max() ** 2, 1e-300)
    for n, (J, K) in enumerate(zip(rows, bcol)):
        u = Bfull.get((I, J), np.zeros((64, 64)))[a]
        v = Bfull.get((I, int(K)), np.zeros((64, 64)))[a]
        assert np.max(np.abs(C[n] - np.outer(u, v))) <= 1e-13 * peak
    n1 = np.random.default_rng(2).uniform(0.5, 2, g.npix)
    n2 = np.random.default_rng(3).uniform(0.5, 2, g.npix)
    C1 = run_BtNB(g, lmax64["kb"], dev(n1), "fp64")
    C2 = run_BtNB(g, lmax64["kb"], dev(n2), "fp64")
    C12 = run_BtNB(g, lmax64["kb"], dev(2.5 * n1 - 0.5 * n2), "fp64")
    assert torch.max(torch.abs(C12 - (2.5 * C1 - 0.5 * C2))).item() <= 1e-13 * torch.max(torch.abs(C12)).item()


def test_lmax64_errors_through_the_abi(lmax64):
    g, kb = lmax64["g"], lmax64["kb"]
    n = dev(lmax64["ninv"])
    bad = torch.empty(g.out_len - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(sp.SympixError) as e:
        sp.sample_BtNB(g, kb, n, bad, "fp64")
    assert e.value.code == "ESIZE"
    with pytest.raises(sp.SympixError) as e:
        sp.sample_D(g, kb, bad)
    assert e.value.code == "ESIZE"
    out = torch.empty(g.out_len, dtype=torch.float64, device="cuda")
    with pytest.raises(sp.SympixError) as e:
        sp.sample_BtNB(g, kb, n[:-1], out, "fp64")
    assert e.value.code == "ESIZE"
    other = sp.Grid(100, 8)
    with pytest.raises(sp.SympixError) as e:
        sp.sample_D(other, kb, torch.empty(other.out_len, dtype=torch.float64, device="cuda"))
    assert e.value.code == "EINVAL"
    with pytest.raises(sp.SympixError) as e:
        sp.sample_BtNB(g, kb, n, out, 7)
    assert e.value.code == "EINVAL"
    # output overlapping N^-1: one buffer holding both, 32-byte aligned
    shared = torch.zeros(g.out_len + g.npix + 4, dtype=torch.float64, device="cuda")
    off = (-(shared.data_ptr() // 8)) % 4
    n_in = shared[off:off + g.npix]
    n_in.copy_(n)
    with pytest.raises(sp.SympixError) as e:
        sp.sample_BtNB(g, kb, n_in, shared[off + g.npix - 2:off + g.npix - 2 + g.out_len], "fp64")
    assert e.value.code == "EINVAL"
    k4 = sp.Grid(40, 4)
    kk = sp.Kernel(k4, np.ones(41), 0.0)
    with pytest.raises(sp.SympixError) as e:
        sp.sample_D(k4, kk, torch.empty(k4.out_len, dtype=torch.float64, device="cuda"))
    assert e.value.code == "EUNSUPPORTED"


# --- transition grid, lmax 256 (tile counts 27, 54, 72: ratios 2 and 4/3) -----

def test_transition_grid_all_blocks():
    lmax = 256
    og = G.make_grid(lmax, 8)
    g = sp.Grid(lmax, 8)
    rng = np.random.default_rng(9)
    ninv = rng.uniform(0.5, 2.0, g.npix)
    ninv[rng.random(g.npix) < 0.1] = 0.0
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    pairs = stored_pairs(og)
    rows = [J for J, _ in pairs]
    say(f"[t256] npix={g.npix} nblocks={g.nblocks} tiles={og.tiles_north[:8]}")
    kb = sp.Kernel(g, b_l, R)
    Cref = O.sample_BtNB(og, b_l, ninv, R, pairs)
    for prec in ("fp64", "fp32", "bf16x6", "bf16x3"):
        C = run_BtNB(g, kb, dev(ninv), prec).cpu().numpy()
        rep = error_report(C, Cref, rows)
        say(f"[t256] BtNB {prec}: {rep}")
        assert rep["gate"] <= GATE[prec]
    kd = sp.Kernel(g, S.prior(lmax), 0.0)
    D = run_D(g, kd).cpu().numpy()
    Dref = O.sample_D(og, S.prior(lmax), None, pairs)
    rep = error_report(D, Dref, rows)
    say(f"[t256] D fp64: {rep}")
    assert rep["gate"] <= GATE["fp64"]


# --- degenerate grids: one or two bands per hemisphere, bands of 1-3 tiles ------

@pytest.mark.parametrize("lmax", [1, 7, 8, 15, 16, 40])
def test_tiny_grids_all_blocks(lmax):
    og = G.make_grid(lmax, 8)
    g = sp.Grid(lmax, 8)
    rng = np.random.default_rng(1000 + lmax)
    ninv = rng.uniform(0.5, 2.0, g.npix)
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    pairs = stored_pairs(og)
    rows = [J for J, _ in pairs]
    say(f"[tiny {lmax}] npix={g.npix} nblocks={g.nblocks} tiles={list(og.tiles_north)}")
    kb = sp.Kernel(g, b_l, R)
    Cref = O.sample_BtNB(og, b_l, ninv, R, pairs)
    n_dev = dev(ninv)
    zero = torch.zeros(g.npix, dtype=torch.float64, device="cuda")
    for prec in ("fp64", "fp32", "bf16x6", "bf16x3"):
        C = run_BtNB(g, kb, n_dev, prec).cpu().numpy()
        rep = error_report(C, Cref, rows)
        say(f"[tiny {lmax}] BtNB {prec}: {rep}")
        assert rep["gate"] <= GATE[prec]
        # N^-1 = 0 everywhere: every mode returns exact zeros
        Z = run_BtNB(g, kb, zero, prec)
        assert int(torch.count_nonzero(Z)) == 0
    kd = sp.Kernel(g, S.prior(lmax), 0.0)
    D = run_D(g, kd).cpu().numpy()
    Dref = O.sample_D(og, S.prior(lmax), None, pairs)
    rep = error_report(D, Dref, rows)
    say(f"[tiny {lmax}] D fp64: {rep}")
    assert rep["gate"] <= GATE["fp64"]


# --- lmax 512: every block against the oracle ----------------------------------

def test_lmax512_every_block():
    """The lmax 512 workload compared in full: every stored block of
    B^T N^-1 B in all four modes, and of D-hat, against the oracle (35,055
    blocks, 1.15 GB per operator)."""
    cfg = S.CONFIGS["lmax512"]
    og = G.make_grid(cfg.lmax, cfg.k)
    g = sp.Grid(cfg.lmax, cfg.k)
    ninv, b_l, R, d_l = config_inputs(cfg, og)
    brp, bcol = g.blocks()
    idx, pairs = block_index(og, brp, bcol, range(og.ntiles))
    assert np.array_equal(idx, np.arange(g.nblocks))
    jrow = [J for J, _ in pairs]
    op = O.LocalOperator(og, b_l, R)
    Cref = np.stack([O.btnb_block(op, ninv, J, K) for J, K in pairs])
    say(f"[lmax512 full] npix={g.npix} nblocks={g.nblocks}: oracle done")
    n_dev = dev(ninv)
    kb = sp.Kernel(g, b_l, R)
    for prec in ("fp64", "fp32", "bf16x6", "bf16x3"):
        C = run_BtNB(g, kb, n_dev, prec).cpu().numpy()
        rep = error_report(C, Cref, jrow)
        say(f"[lmax512 full] BtNB {prec}: {rep}")
        assert rep["gate"] <= GATE[prec]
        del C
        torch.cuda.empty_cache()
    del Cref
    Dref = O.sample_D(og, d_l, None, pairs)
    D = run_D(g, sp.Kernel(g, d_l, 0.0)).cpu().numpy()
    rep = error_report(D, Dref, jrow)
    say(f"[lmax512 full] D fp64: {rep}")
    assert rep["gate"] <= GATE["fp64"]
    torch.cuda.empty_cache()


# --- full-size configurations, sampled block-rows ------------------------------

@pytest.mark.parametrize("name,modes,n_random", [("lmax1500", ("fp64", "fp32", "bf16x6", "bf16x3"), 16),
                                                 ("lmax3000", ("fp64", "fp32", "bf16x6", "bf16x3"), 12)])
def test_full_size_sampled(name, modes, n_random):
    cfg = S.CONFIGS[name]
    og = G.make_grid(cfg.lmax, cfg.k)
    g = sp.Grid(cfg.lmax, cfg.k)
    ninv, b_l, R, d_l = config_inputs(cfg, og)
    rows = sample_rows(og, n_random, seed=cfg.seed)
    brp, bcol = g.blocks()
    idx, pairs = block_index(og, brp, bcol, rows)
    jrow = [J for J, _ in pairs]
    say(f"[{name}] npix={g.npix} nblocks={g.nblocks} sampled rows={len(rows)} blocks={len(idx)}")
    kb = sp.Kernel(g, b_l, R)
    kd = sp.Kernel(g, d_l, 0.0)
    op = O.LocalOperator(og, b_l, R)
    Cref = np.stack([O.btnb_block(op, ninv, J, K) for J, K in pairs])
    idx_t = torch.as_tensor(idx, device="cuda")
    n_dev = dev(ninv)
    for prec in modes:
        C = run_BtNB(g, kb, n_dev, prec)[idx_t].cpu().numpy()
        rep = error_report(C, Cref, jrow)
        say(f"[{name}] BtNB {prec}: {rep}")
        assert rep["gate"] <= GATE[prec]
        del C
        torch.cuda.empty_cache()
    Dref = O.sample_D(og, d_l, None, pairs)
    D = run_D(g, kd)[idx_t].cpu().numpy()
    rep = error_report(D, Dref, jrow)
    say(f"[{name}] D fp64: {rep}")
    assert rep["gate"] <= GATE["fp64"]
    torch.cuda.empty_cache()


# --- the two-hop pattern: every nonzero block of the product -------------------

def two_hop_index(g):
    """Per one-hop stored block, its position in the two-hop output."""
    rp1, col1 = g.pattern_blocks("one_hop")
    rp2, col2 = g.pattern_blocks("two_hop")
    idx = []
    for J in range(g.ntiles):
        row = col2[rp2[J]:rp2[J + 1]]
        pos = np.searchsorted(row, col1[rp1[J]:rp1[J + 1]])
        assert np.array_equal(row[pos], col1[rp1[J]:rp1[J + 1]])
        idx.extend((rp2[J] + pos).tolist())
    return np.asarray(idx, dtype=np.int64)


@pytest.mark.parametrize("lmax", [1, 16, 64, 256])
def test_two_hop_pattern_all_blocks(lmax):
    """Every two-hop block against the oracle in all modes; the blocks the
    one-hop pattern also holds are bitwise equal to sample_BtNB's."""
    og = G.make_grid(lmax, 8)
    g = sp.Grid(lmax, 8)
    rng = np.random.default_rng(2000 + lmax)
    ninv = rng.uniform(0.5, 2.0, g.npix)
    ninv[rng.random(g.npix) < 0.1] = 0.0
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    pairs = O.two_hop_block_list(og)
    rows = [J for J, _ in pairs]
    n2 = len(pairs)
    say(f"[two-hop {lmax}] blocks: one-hop {g.nblocks}, two-hop {n2}")
    kb = sp.Kernel(g, b_l, R)
    Cref = O.sample_BtNB(og, b_l, ninv, R, pairs)
    n_dev = dev(ninv)
    idx = torch.as_tensor(two_hop_index(g), device="cuda")
    for prec in ("fp64", "fp32", "bf16x6", "bf16x3"):
        out = torch.full((n2 * 4096,), float("nan"), dtype=torch.float64, device="cuda")
        sp.sample_BtNB_pattern(g, kb, n_dev, out, prec, "two_hop")
        torch.cuda.synchronize()
        C = out.view(n2, 64, 64)
        rep = error_report(C.cpu().numpy(), Cref, rows)
        say(f"[two-hop {lmax}] {prec}: {rep}")
        assert rep["gate"] <= GATE[prec]
        one = run_BtNB(g, kb, n_dev, prec)
        assert torch.equal(C[idx], one), f"lmax {lmax} {prec}: one-hop blocks differ from sample_BtNB"


def test_two_hop_pattern_full_size_sampled():
    cfg = S.CONFIGS["lmax1500"]
    og = G.make_grid(cfg.lmax, cfg.k)
    g = sp.Grid(cfg.lmax, cfg.k)
    ninv, b_l, R, _ = config_inputs(cfg, og)
    rp, col = g.pattern_blocks("two_hop")
    n2 = len(col)
    rows = sample_rows(og, 8, seed=cfg.seed + 2)
    pairs, idx = [], []
    for J in rows:
        for n in range(rp[J], rp[J + 1]):
            pairs.append((J, int(col[n])))
            idx.append(n)
    say(f"[two-hop {cfg.lmax}] blocks: one-hop {g.nblocks}, two-hop {n2}; sampled {len(pairs)}")
    kb = sp.Kernel(g, b_l, R)
    op = O.LocalOperator(og, b_l, R)
    Cref = np.stack([O.btnb_block(op, ninv, J, K) for J, K in pairs])
    n_dev = dev(ninv)
    idx_t = torch.as_tensor(idx, device="cuda")
    for prec in ("fp64", "bf16x6"):
        out = torch.full((n2 * 4096,), float("nan"), dtype=torch.float64, device="cuda")
        sp.sample_BtNB_pattern(g, kb, n_dev, out, prec, "two_hop")
        torch.cuda.synchronize()
        assert not bool(torch.isnan(out).any()), f"{prec}: a two-hop block was not written"
        rep = error_report(out.view(n2, 64, 64)[idx_t].cpu().numpy(), Cref, [J for J, _ in pairs])
        say(f"[two-hop {cfg.lmax}] {prec}: {rep}")
        assert rep["gate"] <= GATE[prec]
        del out
        torch.cuda.empty_cache()


def test_two_hop_pattern_errors(lmax64):
    g, kb = lmax64["g"], lmax64["kb"]
    n = dev(lmax64["ninv"])
    rp, col = g.pattern_blocks("two_hop")
    out = torch.empty(len(col) * 4096, dtype=torch.float64, device="cuda")
    with pytest.raises(sp.SympixError) as e:
        sp.sample_BtNB_pattern(g, kb, n, out, "fp64", 2)
    assert e.value.code == "EINVAL"
    with pytest.raises(sp.SympixError) as e:
        sp.sample_BtNB_pattern(g, kb, n, out[:-4096], "fp64", "two_hop")
    assert e.value.code == "ESIZE"
    with pytest.raises(sp.SympixError) as e:                      # the one-hop length for the two-hop call
        sp.sample_BtNB_pattern(g, kb, n, out[:g.out_len], "fp64", "two_hop")
    assert e.value.code == "ESIZE"


# --- pixel-domain convolution g = B-hat f (Section 4.1) --------------------------

def run_convolve(g, kern, f_dev):
    out = torch.empty(g.npix, dtype=torch.float64, device="cuda")
    sp.convolve(g, kern, f_dev, out)
    torch.cuda.synchronize()
    return out


def conv_gate(got, ref):
    """max |got - ref| / max |ref| (infinite on any non-finite value)."""
    if not (np.isfinite(got).all() and np.isfinite(ref).all()):
        return float("inf")
    return float(np.abs(got - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("lmax", [1, 8, 16, 40, 64, 256])
def test_convolution_every_tile(lmax):
    og = G.make_grid(lmax, 8)
    g = sp.Grid(lmax, 8)
    rng = np.random.default_rng(2000 + lmax)
    f = rng.standard_normal(g.npix)
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    kb = sp.Kernel(g, b_l, R)
    f_dev = dev(f)
    got = run_convolve(g, kb, f_dev).cpu().numpy().reshape(-1, 64)
    ref = O.convolve(og, b_l, f, R)
    gate = conv_gate(got, ref)
    say(f"[conv {lmax}] npix={g.npix} gate {gate:.3e}")
    assert gate <= GATE["fp64"]
    again = run_convolve(g, kb, f_dev).cpu().numpy().reshape(-1, 64)
    assert np.array_equal(got, again)             # bitwise reproducible


def test_convolution_full_size_sampled():
    cfg = S.CONFIGS["lmax3000"]
    og = G.make_grid(cfg.lmax, cfg.k)
    g = sp.Grid(cfg.lmax, cfg.k)
    rng = np.random.default_rng(4040)
    f = rng.standard_normal(g.npix)
    b_l, R = S.gaussian_beam(cfg.lmax, g.npix, cfg.fwhm_pix)
    kb = sp.Kernel(g, b_l, R)
    got = run_convolve(g, kb, dev(f)).cpu().numpy().reshape(-1, 64)
    tiles = sample_rows(og, 48, seed=cfg.seed)
    ref = O.convolve(og, b_l, f, R, tiles=tiles)
    gate = conv_gate(got[tiles], ref)
    say(f"[conv lmax3000] {len(tiles)} sampled tiles, gate {gate:.3e}")
    assert gate <= GATE["fp64"]
    assert np.isfinite(got).all()


def test_convolution_errors(lmax64):
    g, kb = lmax64["g"], lmax64["kb"]
    f = torch.zeros(g.npix, dtype=torch.float64, device="cuda")
    short = torch.zeros(g.npix - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(sp.SympixError) as ei:
        sp.convolve(g, kb, f, short)
    assert ei.value.code == "ESIZE"
    with pytest.raises(sp.SympixError) as ei:
        sp.convolve(g, kb, f, f)
    assert ei.value.code == "EINVAL"
