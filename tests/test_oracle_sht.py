"""Pins for the oracle's spherical harmonic transforms on the SymPix geometry
(oracle.sht) and the degrade of Eq. 14: lambda_lm against scipy's associated
Legendre functions and against mpmath in extended precision (deep in the range
where the recurrence must rescale), closed forms of the lowest degrees, the
addition theorem for the real basis, synthesis against a dense matrix of
scipy's complex harmonics, the exactness of analysis after synthesis on a grid
whose rings all hold more than 2 L samples (Gauss-Legendre quadrature in
theta, discrete orthogonality in phi), the transpose relation between
synthesis and adjoint, and the degrade against dense matrices."""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as ss

from oracle import grid as G
from oracle import sht as H


def real_basis_dense(lmax, theta, phi):
    """Dense real-harmonic matrix [npts, (lmax+1)^2] from scipy's complex
    harmonics: Y_{l,m} = sqrt(2) (-1)^m Re Y_l^m, Y_{l,-m} = sqrt(2) (-1)^m Im Y_l^m
    (the (-1)^m removes scipy's Condon-Shortley phase)."""
    out = np.zeros((theta.size, (lmax + 1) ** 2))
    for l in range(lmax + 1):
        for m in range(l + 1):
            y = ss.sph_harm_y(l, m, theta, phi)
            if m == 0:
                out[:, l * l + l] = y.real
            else:
                out[:, l * l + l + m] = math.sqrt(2.0) * (-1) ** m * y.real
                out[:, l * l + l - m] = math.sqrt(2.0) * (-1) ** m * y.imag
    return out


def test_lambda_against_scipy_lpmv():
    """scipy evaluates P_l^m from x = cos(theta), so its sqrt(1 - x^2) carries a
    relative error of about eps / sin^2(theta) near the poles (the oracle uses
    sin(theta) itself); the tolerance is that bound plus 1e-12."""
    lmax = 30
    theta = np.array([1e-3, 0.05, 0.7, 1.3, math.pi / 2, 2.2, math.pi - 0.02])
    rtol = 1e-12 + 4e-16 / np.sin(theta) ** 2
    lam = H.lambda_table(lmax, theta)
    for l in range(lmax + 1):
        for m in range(l + 1):
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.exp(math.lgamma(l - m + 1) - math.lgamma(l + m + 1)))
            ref = (-1) ** m * norm * ss.lpmv(m, l, np.cos(theta))
            assert np.all(np.abs(lam[l, m] - ref) <= rtol * np.abs(ref) + 1e-14), (l, m)


@pytest.mark.parametrize("l,m,theta", [(200, 150, 0.05), (400, 390, 0.3), (300, 10, 0.002),
                                        (512, 300, 0.9), (256, 256, 0.01)])
def test_lambda_against_mpmath_through_the_rescaling(l, m, theta):
    """Values far below the double range at l = m (sin^m theta underflows)
    that the rescaled recurrence must still carry correctly."""
    lam = H.lambda_table(l, np.array([theta]))[l, m, 0]
    # P_l^m(x) = (1 - x^2)^(m/2) d^m/dx^m P_l(x) from Rodrigues' formula as an
    # explicit power series, summed with enough digits to absorb its cancellation
    with mpmath.workdps(3 * l + 50):
        th = mpmath.mpf(theta)
        x = mpmath.cos(th)
        series = mpmath.fsum((-1) ** k * mpmath.binomial(l, k) * mpmath.factorial(2 * l - 2 * k)
                             / mpmath.factorial(l - 2 * k - m) * x ** (l - 2 * k - m)
                             for k in range((l - m) // 2 + 1))
        plm = mpmath.sin(th) ** m * series / (mpmath.mpf(2) ** l * mpmath.factorial(l))
        norm = mpmath.sqrt((2 * l + 1) / (4 * mpmath.pi) * mpmath.factorial(l - m) / mpmath.factorial(l + m))
        ref = float(norm * plm)
    if abs(ref) < 1e-300:
        assert abs(lam) < 1e-290
    else:
        assert abs(lam - ref) <= 1e-12 * abs(ref), (lam, ref)


def test_lowest_degrees_closed_forms():
    th = np.linspace(0.01, math.pi - 0.01, 23)
    lam = H.lambda_table(2, th)
    c, s = np.cos(th), np.sin(th)
    assert np.allclose(lam[0, 0], 1 / math.sqrt(4 * math.pi), rtol=1e-15)
    assert np.allclose(lam[1, 0], math.sqrt(3 / (4 * math.pi)) * c, rtol=1e-14, atol=1e-16)
    assert np.allclose(lam[1, 1], math.sqrt(3 / (8 * math.pi)) * s, rtol=1e-14)
    assert np.allclose(lam[2, 0], math.sqrt(5 / (16 * math.pi)) * (3 * c * c - 1), rtol=1e-13, atol=1e-15)
    assert np.allclose(lam[2, 2], math.sqrt(15 / (32 * math.pi)) * s * s, rtol=1e-13)


def test_addition_theorem_real_basis():
    """sum_m Y_lm(n1) Y_lm(n2) = (2l+1)/(4 pi) P_l(n1 . n2) for the real basis."""
    rng = np.random.default_rng(3)
    lmax = 40
    th = rng.uniform(0, math.pi, 6)
    ph = rng.uniform(0, 2 * math.pi, 6)
    lam = H.lambda_table(lmax, th)
    for i in range(3):
        a, b = 2 * i, 2 * i + 1
        cosg = (math.cos(th[a]) * math.cos(th[b]) + math.sin(th[a]) * math.sin(th[b]) * math.cos(ph[a] - ph[b]))
        for l in range(lmax + 1):
            acc = lam[l, 0, a] * lam[l, 0, b]
            for m in range(1, l + 1):
                acc += 2 * lam[l, m, a] * lam[l, m, b] * (math.cos(m * ph[a]) * math.cos(m * ph[b]) +
                                                            math.sin(m * ph[a]) * math.sin(m * ph[b]))
            ref = (2 * l + 1) / (4 * math.pi) * ss.eval_legendre(l, cosg)
            assert abs(acc - ref) <= 1e-12 * (2 * l + 1), (l, acc, ref)


@pytest.mark.parametrize("lmax,L", [(16, 10), (24, 24)])
def test_synthesis_matches_dense_scipy_harmonics(lmax, L):
    g = G.make_grid(lmax, 2)
    ring, pin, nr, phi = g.pixel_coords()
    Yd = real_basis_dense(L, g.theta[ring], phi)
    rng = np.random.default_rng(lmax)
    a = rng.standard_normal((L + 1) ** 2)
    f = H.synthesis(g, a, L)
    assert np.abs(f - Yd @ a).max() <= 1e-12 * np.abs(Yd @ a).max()
    x = rng.standard_normal(g.npix)
    assert np.abs(H.adjoint(g, x, L) - Yd.T @ x).max() <= 1e-12 * np.abs(Yd.T @ x).max()


def test_analysis_inverts_synthesis_when_every_ring_is_long_enough():
    """lmax 64, k = 8: every ring holds 144 > 2 L pixels for L = 64 and the 80
    Gauss-Legendre rings integrate degree <= 159 exactly, so Y^T W Y = I."""
    g = G.make_grid(64, 8)
    assert min(g.ring_npix()) > 2 * 64
    rng = np.random.default_rng(11)
    a = rng.standard_normal(65 ** 2)
    back = H.analysis(g, H.synthesis(g, a, 64), 64)
    assert np.abs(back - a).max() <= 1e-12


def test_quadrature_weights_sum_to_the_sphere():
    g = G.make_grid(40, 4)
    assert abs(H.pixel_weights(g).sum() - 4 * math.pi) <= 1e-12


def test_adjoint_is_the_transpose_of_synthesis():
    g = G.make_grid(48, 4)
    L = 40
    rng = np.random.default_rng(5)
    a = rng.standard_normal((L + 1) ** 2)
    f = rng.standard_normal(g.npix)
    lhs = H.synthesis(g, a, L) @ f
    rhs = a @ H.adjoint(g, f, L)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_polar_cut_keeps_the_round_trip_exact():
    """The polar rings of a SymPix grid hold fewer than 2 L + 1 pixels, but the
    cut of Eq. 3 only drops modes that are negligible there: on this library's
    grid analysis after synthesis still returns the coefficients to ~1e-13 at
    L = lmax (the paper's Table 1 reports 7.8e-3 for its own, smaller grids)."""
    g = G.make_grid(128, 8)
    assert min(g.ring_npix()) < 2 * 128 + 1
    rng = np.random.default_rng(2)
    a = rng.standard_normal(129 ** 2)
    back = H.analysis(g, H.synthesis(g, a, 128), 128)
    assert np.abs(back - a).max() <= 1e-12


def test_degrade_matches_dense_matrices():
    g_obs = G.make_grid(20, 2)
    g2 = G.make_grid(12, 2)
    L = 12
    ro, po, no, pho = g_obs.pixel_coords()
    r2, p2, n2, ph2 = g2.pixel_coords()
    Yo = real_basis_dense(L, g_obs.theta[ro], pho)
    Y2 = real_basis_dense(L, g2.theta[r2], ph2)
    w2 = g2.weight[r2] * 2 * math.pi / n2
    rng = np.random.default_rng(9)
    th = rng.uniform(0.5, 2.0, g_obs.npix)
    ref = w2 * (Y2 @ (Yo.T @ th))
    got = H.degrade(g_obs, g2, th, L)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_lambda_m_is_the_tables_column():
    """One order's column (lambda_m, for band limits where the whole table
    is too large) takes the same steps as lambda_table: equal bit for bit."""
    th = np.array([0.003, 0.4, 1.1, 1.5707, 2.9])
    tab = H.lambda_table(60, th)
    for m in (0, 1, 7, 31, 60):
        np.testing.assert_array_equal(H.lambda_m(60, m, th), tab[m:, m, :])


def test_lambda_m_where_lambda_mm_is_below_the_double_range():
    """At m = 1000 and sin(theta) = 0.45, lambda_mm ~ 1e-336 lies below the
    smallest double, yet lambda_lm is of order one by l = 2400 (past the
    turning point l ~ m / sin(theta)): against mpmath's Rodrigues series."""
    m, theta = 1000, math.asin(0.45)
    col = H.lambda_m(2400, m, np.array([theta]))[:, 0]
    assert abs(col[0]) == 0.0                          # below 2^-1074
    for l in (2300, 2400):
        with mpmath.workdps(3 * l + 50):
            th = mpmath.mpf(theta)
            x = mpmath.cos(th)
            series = mpmath.fsum((-1) ** k * mpmath.binomial(l, k) * mpmath.factorial(2 * l - 2 * k)
                                 / mpmath.factorial(l - 2 * k - m) * x ** (l - 2 * k - m)
                                 for k in range((l - m) // 2 + 1))
            plm = mpmath.sin(th) ** m * series / (mpmath.mpf(2) ** l * mpmath.factorial(l))
            norm = mpmath.sqrt((2 * l + 1) / (4 * mpmath.pi) * mpmath.factorial(l - m) / mpmath.factorial(l + m))
            ref = float(norm * plm)
        assert abs(ref) > 1e-3
        assert abs(col[l - m] - ref) <= 1e-11 * abs(ref), (l, col[l - m], ref)


def test_synthesis_on_chosen_rings_is_the_full_maps_restriction():
    """The ring-restricted synthesis (used to check the device transform at
    full size on a few rings) gives exactly the full map's values there."""
    g = G.make_grid(40, 4)
    L = 40
    a = np.random.default_rng(12).standard_normal((L + 1) ** 2)
    full = H.synthesis(g, a, L)
    ring, _, _, _ = g.pixel_coords()
    rings = [0, 7, g.nrings // 2, g.nrings - 1]
    part = H.synthesis(g, a, L, rings=rings)
    assert np.array_equal(part, full[np.isin(ring, rings)])
