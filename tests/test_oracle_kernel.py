"""Pins for the oracle's kernel b(x) = sum_l (2l+1)/(4 pi) b_l P_l(x) (Eq. 10)."""
import mpmath
import numpy as np
import pytest
import scipy.special as ss

from oracle.kernel import legendre_series_in_x, legendre_series_in_y


def test_addition_theorem_against_spherical_harmonics():
    """Eq. 10 is the addition theorem: sum_l b_l sum_m Y_lm(n1) Y*_lm(n2) = b(n1.n2)."""
    rng = np.random.default_rng(5)
    for lmax in (0, 1, 3, 10):
        b_l = rng.uniform(-1.0, 2.0, lmax + 1)
        th1, th2 = rng.uniform(0, np.pi, 2)
        ph1, ph2 = rng.uniform(0, 2 * np.pi, 2)
        ref = 0.0
        for l in range(lmax + 1):
            for m in range(-l, l + 1):
                ref += b_l[l] * (ss.sph_harm_y(l, m, th1, ph1) * np.conj(ss.sph_harm_y(l, m, th2, ph2))).real
        cosg = np.cos(th1) * np.cos(th2) + np.sin(th1) * np.sin(th2) * np.cos(ph1 - ph2)
        y = 1.0 - cosg
        assert abs(legendre_series_in_y(b_l, y) - ref) < 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("L", [1, 7, 64, 512, 3000])
def test_christoffel_darboux_closed_form(L):
    """b_l = 1 for all l: 4 pi b(x) = (L+1)(P_L(x) - P_{L+1}(x)) / (1 - x), and (L+1)^2 at x = 1."""
    b_l = np.ones(L + 1)
    x = np.array([-0.99, -0.3, 0.0, 0.41, 0.9, 0.999])
    ref = (L + 1) * (ss.eval_legendre(L, x) - ss.eval_legendre(L + 1, x)) / (1.0 - x)
    got = 4 * np.pi * legendre_series_in_y(b_l, 1.0 - x)
    assert np.max(np.abs(got - ref)) < 1e-11 * (L + 1) ** 2
    assert abs(4 * np.pi * legendre_series_in_y(b_l, np.array([0.0]))[0] - (L + 1) ** 2) < 1e-12 * (L + 1) ** 2


@pytest.mark.parametrize("L", [0, 2, 13, 200])
def test_single_multipole_is_legendre_polynomial(L):
    b_l = np.zeros(L + 1)
    b_l[L] = 1.0
    x = np.linspace(-1, 1, 41)
    got = 4 * np.pi / (2 * L + 1) * legendre_series_in_y(b_l, 1.0 - x)
    assert np.max(np.abs(got - ss.eval_legendre(L, x))) < 1e-13


def test_y_and_x_recurrences_agree_away_from_the_pole():
    lmax = 3000
    ell = np.arange(lmax + 1.0)
    for b_l in (np.exp(-0.5 * ell * (ell + 1) * 1.3e-3 ** 2), (ell + 1.0) ** 2):
        y = np.linspace(0.1, 2.0, 25)
        a = legendre_series_in_y(b_l, y)
        b = legendre_series_in_x(b_l, 1.0 - y)
        peak = legendre_series_in_y(b_l, np.array([0.0]))[0]
        assert np.max(np.abs(a - b)) < 1e-14 * peak


def test_small_separation_accuracy_against_50_digit_sum():
    """Pairs a fraction of a pixel apart at lmax = 3000 (y ~ 1e-8 .. 1e-5): the
    sum in y must keep ~1e-14 of the peak, checked against 50-digit arithmetic."""
    lmax = 3000
    mpmath.mp.dps = 50
    ell = np.arange(lmax + 1.0)
    sigma = 1.27e-3
    b_l = np.exp(-0.5 * ell * (ell + 1) * sigma ** 2)
    for coef in (b_l, (ell + 1.0) ** 2):
        peak = legendre_series_in_y(coef, np.array([0.0]))[0]
        for y in (1e-8, 3e-7, 4e-6):
            x = 1 - mpmath.mpf(y)
            p0, p1 = mpmath.mpf(1), x
            acc = mpmath.mpf(coef[0]) * 1 / (4 * mpmath.pi) + 3 * mpmath.mpf(coef[1]) * x / (4 * mpmath.pi)
            for l in range(1, lmax):
                p0, p1 = p1, ((2 * l + 1) * x * p1 - l * p0) / (l + 1)
                acc += (2 * (l + 1) + 1) * mpmath.mpf(coef[l + 1]) * p1 / (4 * mpmath.pi)
            got = legendre_series_in_y(coef, np.array([y]))[0]
            assert abs(got - float(acc)) < 2e-14 * peak
