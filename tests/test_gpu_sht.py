"""GPU parity of the spherical harmonic transforms on the SymPix geometry
(Eq. 1) and the degrade of Eq. 14 through the C ABI, against the FP64 oracle
(oracle.sht): every pixel and coefficient on small grids (several tile sizes,
band limits below and at the grid's lmax), the degrade between two grids,
sampled rings at lmax 512, and at the full sizes (lmax 1500 and 3000) the
properties that hold at any size: analysis inverts synthesis on this library's
grids (to the level the oracle shows at lmax 128 and 512) and Y^T is the
transpose of Y (<Y a, f> = <a, Y^T f>)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1504_04653_amd as sp
from oracle import grid as G
from oracle import sht as H

pytestmark = pytest.mark.gpu

TOL = 1e-12          # FP64 both sides; FFT against direct sums, relative to the largest value


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


def rel(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


# (lmax, k, L); k = 3 at lmax 38 gives rings of odd length (81 pixels), which
# take the ring FFT at full length, every other ring at half length
CASES = [(16, 2, 16), (40, 4, 30), (64, 8, 64), (128, 8, 128), (100, 8, 60), (38, 3, 38),
         (16, 2, 0), (32, 4, 48)]                         # L = 0; L above the grid's lmax (modes alias)


@pytest.mark.parametrize("lmax,k,L", CASES)
def test_transforms_against_oracle(lmax, k, L):
    og, g = G.make_grid(lmax, k), sp.Grid(lmax, k)
    s = sp.Sht(g, L)
    rng = np.random.default_rng(lmax + 7 * k + L)
    a = rng.standard_normal((L + 1) ** 2)
    f = rng.standard_normal(g.npix)
    out_map = torch.full((g.npix,), float("nan"), dtype=torch.float64, device="cuda")
    out_alm = torch.full(((L + 1) ** 2,), float("nan"), dtype=torch.float64, device="cuda")
    s.synthesis(dev(a), out_map)
    torch.cuda.synchronize()
    e_syn = rel(out_map.cpu().numpy(), H.synthesis(og, a, L))
    s.adjoint(dev(f), out_alm)
    torch.cuda.synchronize()
    e_adj = rel(out_alm.cpu().numpy(), H.adjoint(og, f, L))
    s.analysis(dev(f), out_alm)
    torch.cuda.synchronize()
    e_ana = rel(out_alm.cpu().numpy(), H.analysis(og, f, L))
    say(f"[sht lmax={lmax} k={k} L={L}] npix={g.npix} synthesis {e_syn:.2e} adjoint {e_adj:.2e} analysis {e_ana:.2e}")
    assert max(e_syn, e_adj, e_ana) <= TOL


@pytest.mark.parametrize("obs,target,L", [((64, 8), (32, 4), 32), ((48, 4), (64, 8), 40)])
def test_degrade_against_oracle(obs, target, L):
    og_o, og_t = G.make_grid(*obs), G.make_grid(*target)
    g_o, g_t = sp.Grid(*obs), sp.Grid(*target)
    s_o, s_t = sp.Sht(g_o, L), sp.Sht(g_t, L)
    rng = np.random.default_rng(L)
    th = rng.uniform(0.5, 2.0, g_o.npix)
    th[rng.random(g_o.npix) < 0.2] = 0.0                # masked pixels
    out = torch.full((g_t.npix,), float("nan"), dtype=torch.float64, device="cuda")
    sp.degrade(s_o, s_t, dev(th), out)
    torch.cuda.synchronize()
    e = rel(out.cpu().numpy(), H.degrade(og_o, og_t, th, L))
    say(f"[degrade {obs} -> {target} L={L}] {e:.2e}")
    assert e <= TOL


def test_sampled_rings_at_lmax512():
    """Synthesis on every pixel of two polar and two equatorial rings, and
    analysis of a band-limited map, against the oracle at lmax 512."""
    lmax = L = 512
    og, g = G.make_grid(lmax, 8), sp.Grid(lmax, 8)
    s = sp.Sht(g, L)
    rng = np.random.default_rng(512)
    a = rng.standard_normal((L + 1) ** 2) / np.sqrt(np.repeat(np.arange(L + 1), 2 * np.arange(L + 1) + 1) + 1.0)
    out = torch.empty(g.npix, dtype=torch.float64, device="cuda")
    s.synthesis(dev(a), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ring, pin, nr, phi = og.pixel_coords()
    rings = [0, 5, og.nrings // 2 - 1, og.nrings - 3]
    lam = H.lambda_table(L, og.theta[rings])
    worst = 0.0
    for q, r in enumerate(rings):
        pix = np.nonzero(ring == r)[0]
        ref = np.zeros(pix.size)
        for m in range(L + 1):
            ls = np.arange(m, L + 1)
            Fc = a[ls * ls + ls + m] @ lam[m:, m, q]
            if m == 0:
                ref += Fc
            else:
                Fs = a[ls * ls + ls - m] @ lam[m:, m, q]
                ref += np.sqrt(2.0) * (Fc * np.cos(m * phi[pix]) + Fs * np.sin(m * phi[pix]))
        worst = max(worst, np.abs(got[pix] - ref).max() / np.abs(got).max())
    back = torch.empty((L + 1) ** 2, dtype=torch.float64, device="cuda")
    s.analysis(out, back)
    torch.cuda.synchronize()
    e_rt = float(np.abs(back.cpu().numpy() - a).max() / np.abs(a).max())
    say(f"[sht lmax=512] sampled rings {worst:.2e}, analysis of the synthesised map {e_rt:.2e}")
    assert worst <= TOL
    assert e_rt <= 1e-11


@pytest.mark.parametrize("lmax", [1500, 3000])
def test_full_size_round_trip_and_transpose(lmax):
    L = lmax
    g = sp.Grid(lmax, 8)
    s = sp.Sht(g, L)
    rng = np.random.default_rng(lmax)
    ell = np.repeat(np.arange(L + 1), 2 * np.arange(L + 1) + 1)
    a = dev(rng.standard_normal((L + 1) ** 2) / np.sqrt(ell + 1.0))
    f = torch.empty(g.npix, dtype=torch.float64, device="cuda")
    back = torch.empty_like(a)
    s.synthesis(a, f)
    s.analysis(f, back)
    torch.cuda.synchronize()
    e_rt = float((back - a).abs().max() / a.abs().max())
    x = dev(rng.standard_normal(g.npix))
    yt = torch.empty_like(a)
    s.adjoint(x, yt)
    torch.cuda.synchronize()
    lhs, rhs = float(f @ x), float(a @ yt)
    e_tr = abs(lhs - rhs) / (float(f.abs().sum()) * float(x.abs().max()))
    assert bool(torch.isfinite(f).all()) and bool(torch.isfinite(yt).all())
    say(f"[sht lmax={lmax}] npix={g.npix}: analysis of synthesis {e_rt:.2e}; <Ya,x> vs <a,Y^T x> {e_tr:.2e}")
    assert e_rt <= 1e-10
    assert e_tr <= 1e-12


# (L, orders m whose window [m / L, 10^(-323/m)] of sin(theta) is not empty)
FULL_ORDERS = {2400: (1000, 1100, 1200), 3000: (1200, 1500, 2000)}


@pytest.mark.parametrize("L", [2400, 3000])
def test_orders_whose_lambda_mm_is_below_the_double_range(L):
    """On rings with sin(theta) in [m / L, 10^(-323/m)], lambda_mm of order m
    lies below the smallest double but lambda_lm is of order one before l = L
    (the turning point m / sin(theta) < L).  Transpose of a map that is nonzero
    on such rings (and on a polar and an equatorial ring), and synthesis of
    coefficients of those orders (and of m = 0, 1, L) on the same rings,
    against the oracle's per-order recurrence; at L = 3000 this is the
    workload the SHT bench times (lmax 3000 grid, L = lmax)."""
    lmax = L
    og, g = G.make_grid(lmax, 8), sp.Grid(lmax, 8)
    s = sp.Sht(g, L)
    ring, pin, nr, phi = og.pixel_coords()
    st = np.sin(og.theta[: og.nrings // 2])
    windows = [(m / L + 10.0 ** (-323.0 / m)) / 2 for m in FULL_ORDERS[L]]
    rings = sorted({0, og.nrings // 2 - 1} | {int(np.argmin(np.abs(st - v))) for v in windows})
    orders = sorted({0, 1, L // 2, L} | set(FULL_ORDERS[L]) | {FULL_ORDERS[L][0] - 1})
    lam = {m: H.lambda_m(L, m, og.theta[rings]) for m in orders}      # [l - m, ring]
    for m in FULL_ORDERS[L]:       # the case: some chosen ring has lambda_mm = 0 yet |lambda_lm| ~ 1
        assert any(lam[m][0, q] == 0.0 and np.abs(lam[m][:, q]).max() > 0.1 for q in range(len(rings)))
    rng = np.random.default_rng(L)
    # transpose: x nonzero on the chosen rings only
    x = np.zeros(g.npix)
    on = np.isin(ring, rings)
    x[on] = rng.standard_normal(int(on.sum()))
    yt = torch.empty((L + 1) ** 2, dtype=torch.float64, device="cuda")
    s.adjoint(dev(x), yt)
    torch.cuda.synchronize()
    got = yt.cpu().numpy()
    worst, scale = 0.0, 0.0
    for m in orders:
        ls = np.arange(m, L + 1)
        gc = np.array([np.sum(x[ring == r] * np.cos(m * phi[ring == r])) for r in rings])
        gs = np.array([np.sum(x[ring == r] * np.sin(m * phi[ring == r])) for r in rings])
        ref_c = lam[m] @ gc * (1.0 if m == 0 else np.sqrt(2.0))
        worst = max(worst, np.abs(got[ls * ls + ls + m] - ref_c).max())
        scale = max(scale, np.abs(ref_c).max())
        if m > 0:
            ref_s = np.sqrt(2.0) * (lam[m] @ gs)
            worst = max(worst, np.abs(got[ls * ls + ls - m] - ref_s).max())
    e_adj = worst / scale
    # synthesis of coefficients of the chosen orders, read on the chosen rings
    a = np.zeros((L + 1) ** 2)
    for m in orders:
        ls = np.arange(m, L + 1)
        a[ls * ls + ls + m] = rng.standard_normal(ls.size)
        if m > 0:
            a[ls * ls + ls - m] = rng.standard_normal(ls.size)
    out = torch.empty(g.npix, dtype=torch.float64, device="cuda")
    s.synthesis(dev(a), out)
    torch.cuda.synchronize()
    f = out.cpu().numpy()
    worst, scale = 0.0, 0.0
    for q, r in enumerate(rings):
        pix = np.nonzero(ring == r)[0]
        ref = np.zeros(pix.size)
        for m in orders:
            ls = np.arange(m, L + 1)
            Fc = a[ls * ls + ls + m] @ lam[m][:, q]
            if m == 0:
                ref += Fc
            else:
                Fs = a[ls * ls + ls - m] @ lam[m][:, q]
                ref += np.sqrt(2.0) * (Fc * np.cos(m * phi[pix]) + Fs * np.sin(m * phi[pix]))
        worst = max(worst, np.abs(f[pix] - ref).max())
        scale = max(scale, np.abs(ref).max())
    e_syn = worst / scale
    # Near the pole cos(theta) ~ 1 makes the recurrence's two roots nearly
    # equal, so a rounding error made at step j grows about linearly over the
    # steps after it: random roundings leave about eps L^1.5 (2.6e-11 at L =
    # 2400, 3.6e-11 at 3000; eps = 2^-52) between two orderings of the same FP64
    # recurrence.  Measured: 1.2-1.7e-12 at L = 2400, 2.6-3.6e-12 at 3000, the
    # polar ring at m = 0, 1 (every other ring agrees to 2e-14).
    tol = np.finfo(np.float64).eps * L ** 1.5
    say(f"[sht lmax={L}] rings {rings} orders {orders}: transpose {e_adj:.2e}, synthesis {e_syn:.2e} "
        f"(bound {tol:.1e})")
    assert e_adj <= tol and e_syn <= tol


@pytest.mark.parametrize("lmax,k", [(300, 16), (1000, 4), (700, 5)])
def test_round_trip_and_transpose_other_tile_sizes(lmax, k):
    """Tile sizes other than 8 at larger band limits (k = 5 gives rings of odd
    length, taking the full-length ring FFT): analysis inverts synthesis and
    <Y a, x> = <a, Y^T x>, as at k = 8."""
    L = lmax
    g = sp.Grid(lmax, k)
    s = sp.Sht(g, L)
    rng = np.random.default_rng(lmax + k)
    ell = np.repeat(np.arange(L + 1), 2 * np.arange(L + 1) + 1)
    a = dev(rng.standard_normal((L + 1) ** 2) / np.sqrt(ell + 1.0))
    f = torch.empty(g.npix, dtype=torch.float64, device="cuda")
    back = torch.empty_like(a)
    s.synthesis(a, f)
    s.analysis(f, back)
    x = dev(rng.standard_normal(g.npix))
    yt = torch.empty_like(a)
    s.adjoint(x, yt)
    torch.cuda.synchronize()
    e_rt = float((back - a).abs().max() / a.abs().max())
    e_tr = abs(float(f @ x) - float(a @ yt)) / (float(f.abs().sum()) * float(x.abs().max()))
    say(f"[sht lmax={lmax} k={k}] npix={g.npix}: analysis of synthesis {e_rt:.2e}; <Ya,x> vs <a,Y^T x> {e_tr:.2e}")
    assert e_rt <= 1e-10 and e_tr <= 1e-12


def test_plans_sharing_a_ring_kernel():
    """Two plans whose ring FFTs take the same kernel instantiation but need
    different LDS (odd rings of 6075 and 5625 pixels at k = 5: 97 and 90 KB):
    creating the second plan must not lower the first one's LDS allowance, so
    the first plan's transforms still run after the second exists."""
    ga, gb = sp.Grid(3000, 5), sp.Grid(2700, 5)
    sa = sp.Sht(ga, 3000)
    sb = sp.Sht(gb, 2700)
    for g, s, L in ((ga, sa, 3000), (gb, sb, 2700)):
        rng = np.random.default_rng(L)
        ell = np.repeat(np.arange(L + 1), 2 * np.arange(L + 1) + 1)
        a = dev(rng.standard_normal((L + 1) ** 2) / np.sqrt(ell + 1.0))
        f = torch.empty(g.npix, dtype=torch.float64, device="cuda")
        back = torch.empty_like(a)
        s.synthesis(a, f)
        s.analysis(f, back)
        torch.cuda.synchronize()
        e_rt = float((back - a).abs().max() / a.abs().max())
        say(f"[sht lmax={L} k=5] npix={g.npix}: analysis of synthesis {e_rt:.2e}")
        assert e_rt <= 1e-10


@pytest.mark.parametrize("lmax", [511, 639, 767])
def test_table1_round_trip_on_this_grid(lmax):
    """Table 1's experiment (Section 3.3) on this library's grids: 100 draws of
    unit-Gaussian a_lm at L = lmax, synthesis then analysis, max and mean
    |a_hat - a|.  These grids keep every polar sample the analysis needs (7-15%
    more pixels than Table 1 prints), so the round trip is exact to rounding,
    like Table 1's Gauss-Legendre rows."""
    g = sp.Grid(lmax, 8)
    s = sp.Sht(g, lmax)
    n = (lmax + 1) ** 2
    gen = torch.Generator(device="cuda").manual_seed(lmax)
    f = torch.empty(g.npix, dtype=torch.float64, device="cuda")
    back = torch.empty(n, dtype=torch.float64, device="cuda")
    mx = torch.zeros((), dtype=torch.float64, device="cuda")
    tot = torch.zeros((), dtype=torch.float64, device="cuda")
    for _ in range(100):
        a = torch.randn(n, dtype=torch.float64, device="cuda", generator=gen)
        s.synthesis(a, f)
        s.analysis(f, back)
        e = (back - a).abs()
        mx = torch.maximum(mx, e.max())
        tot += e.sum()
    torch.cuda.synchronize()
    emax, emean = float(mx), float(tot) / (100 * n)
    say(f"[table 1 lmax={lmax}] npix={g.npix}: max {emax:.2e} mean {emean:.2e} over 100 draws")
    assert emax <= 1e-10 and emean <= 1e-12


def test_sht_errors():
    g, g2 = sp.Grid(32, 4), sp.Grid(48, 4)
    s, s2, s3 = sp.Sht(g, 20), sp.Sht(g2, 20), sp.Sht(g2, 24)
    alm = torch.zeros(21 ** 2, dtype=torch.float64, device="cuda")
    m = torch.zeros(g.npix, dtype=torch.float64, device="cuda")
    m2 = torch.zeros(g2.npix, dtype=torch.float64, device="cuda")
    for bad, code in ((lambda: s.synthesis(alm[:-1], m), "ESIZE"),
                      (lambda: s.synthesis(alm, m[:-1]), "ESIZE"),
                      (lambda: s.analysis(m2, alm), "ESIZE"),
                      (lambda: sp.degrade(s, s3, m, m2), "EINVAL"),
                      (lambda: sp.degrade(s, s2, m, m), "ESIZE")):
        with pytest.raises(sp.SympixError) as ei:
            bad()
        assert ei.value.code == code
    with pytest.raises(sp.SympixError) as ei:
        sp.Sht(g, -1)
    assert ei.value.code == "EINVAL"
    with pytest.raises(sp.SympixError) as ei:
        sp.Sht(g, 5000)
    assert ei.value.code == "EUNSUPPORTED"
