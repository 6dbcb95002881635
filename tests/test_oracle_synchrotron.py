"""Pins of the oracle's synchrotron functions (Sec. 3.2.1) against routes that do not
use its integral representation: library Bessel functions, the paper's own series,
closed-form integrals, asymptotic expansions and printed/known values."""
import math

import mpmath as mp
import numpy as np
import pytest

mp.mp.dps = 40


def _G_besselk(x):
    x = mp.mpf(x)
    return x * mp.besselk(mp.mpf(2) / 3, x)


def _int0x_K13_series(x, terms=60):
    """int_0^x K_{1/3} from the I-series of K (Sec. 3.2.1) integrated term by term."""
    x = mp.mpf(x)
    nu = mp.mpf(1) / 3
    s = mp.mpf(0)
    for n in range(terms):
        for sgn, a in ((1, -nu), (-1, nu)):
            # int_0^x (t/2)^{2n+a} dt / (n! Gamma(n+a+1)) = 2 (x/2)^{2n+a+1}/((2n+a+1) n! Gamma(n+a+1))
            s += sgn * 2 * (x / 2) ** (2 * n + a + 1) / ((2 * n + a + 1) * mp.factorial(n) * mp.gamma(n + a + 1))
    return mp.pi / (2 * mp.sin(nu * mp.pi)) * s


def _F_series(x):
    """F = 2G - x int_x^inf K_{1/3} (K_{5/3} = -2 K'_{2/3} - K_{1/3}, DLMF 10.29.1),
    with int_0^inf K_{1/3} = pi/sqrt(3) (DLMF 10.43.19) and the I-series for both
    G (Sec. 3.2.1) and int_0^x K_{1/3}."""
    x = mp.mpf(x)
    nu = mp.mpf(2) / 3
    Ineg = sum((x / 2) ** (2 * n - nu) / (mp.factorial(n) * mp.gamma(n - nu + 1)) for n in range(60))
    Ipos = sum((x / 2) ** (2 * n + nu) / (mp.factorial(n) * mp.gamma(n + nu + 1)) for n in range(60))
    G = x * mp.pi / 2 * (Ineg - Ipos) / mp.sin(nu * mp.pi)
    tail13 = mp.pi / mp.sqrt(3) - _int0x_K13_series(x)
    return 2 * G - x * tail13


def test_G_matches_library_besselk(orc):
    xs = np.concatenate([10.0 ** np.linspace(-8, 2.5, 24), [400.0, 700.0]])
    F, G = orc.synchrotron(xs)
    for x, g in zip(xs, G):
        ref = float(_G_besselk(x))
        assert abs(g / ref - 1) < 5e-14, (x, g, ref)


def test_F_matches_series_route(orc):
    # the series route cancels badly beyond x ~ 10 even at 40 digits; stay below
    xs = 10.0 ** np.linspace(-7, 0.7, 12)
    F, _ = orc.synchrotron(xs)
    for x, f in zip(xs, F):
        ref = float(_F_series(x))
        assert abs(f / ref - 1) < 5e-14, (x, f, ref)


def test_F_matches_library_quadrature_large_x(orc):
    # x int_x^inf K_{5/3} with SciPy's K_nu and adaptive quadrature (scaled by e^x)
    from scipy import integrate, special
    for x in (5.0, 12.0, 30.0, 80.0, 200.0):
        val, err = integrate.quad(lambda s: special.kve(5.0 / 3.0, s) * math.exp(x - s), x, np.inf,
                                  epsabs=0, epsrel=2e-14, limit=200)
        ref = x * val * math.exp(-x)
        F, _ = orc.synchrotron([x])
        assert abs(F[0] / ref - 1) < 1e-12, (x, F[0], ref)


def test_paper_small_x_series_S(orc):
    """S(x) of Sec. 3.2.1 with k = 2 reproduces G for x < 0.001."""
    def S(x, k=2):
        x = mp.mpf(x)
        pre = mp.pi * x / (2 * mp.sin(2 * mp.pi / 3))
        return pre * sum((x / 2) ** (2 * n) / mp.factorial(n) *
                         ((x / 2) ** (-mp.mpf(2) / 3) / mp.gamma(n + mp.mpf(1) / 3) -
                          (x / 2) ** (mp.mpf(2) / 3) / mp.gamma(n + mp.mpf(5) / 3)) for n in range(k + 1))
    xs = [1e-9, 1e-6, 1e-4, 9.9e-4]
    _, G = orc.synchrotron(xs)
    for x, g in zip(xs, G):
        assert abs(g / float(S(x)) - 1) < 5e-15


def _log_trapezoid(f, lo=-40.0, hi=7.0, n=6000):
    s = np.linspace(lo, hi, n)
    x = np.exp(s)
    v = f(x) * x
    return float(np.trapezoid(v, s))


def test_closed_form_integrals(orc):
    F = lambda x: orc.synchrotron(x)[0]
    G = lambda x: orc.synchrotron(x)[1]
    # int_0^inf F = 8 pi / (9 sqrt 3), int_0^inf G = 2 pi / (3 sqrt 3)
    assert abs(_log_trapezoid(F) / (8 * math.pi / (9 * math.sqrt(3))) - 1) < 1e-12
    assert abs(_log_trapezoid(G) / (2 * math.pi / (3 * math.sqrt(3))) - 1) < 1e-12
    # int_0^inf F(x)/x dx = 5 pi / 3 (F/x ~ x^{-2/3} at 0: start far down)
    assert abs(_log_trapezoid(lambda x: F(x) / x, lo=-120.0, n=12000) / (5 * math.pi / 3) - 1) < 1e-12


@pytest.mark.parametrize("mu", [0.5, 2.0, 3.5])
def test_mellin_moments(orc, mu):
    """int x^{mu-1} F = 2^mu/(mu+1) Gamma(mu/2+1/6) Gamma(mu/2+11/6);
    int x^{mu-1} G = 2^{mu-1} Gamma(mu/2+1/6) Gamma(mu/2+5/6)  (Mellin transforms of K_nu)."""
    F = lambda x: orc.synchrotron(x)[0]
    G = lambda x: orc.synchrotron(x)[1]
    refF = 2 ** mu / (mu + 1) * math.gamma(mu / 2 + 1 / 6) * math.gamma(mu / 2 + 11 / 6)
    refG = 2 ** (mu - 1) * math.gamma(mu / 2 + 1 / 6) * math.gamma(mu / 2 + 5 / 6)
    assert abs(_log_trapezoid(lambda x: F(x) * x ** (mu - 1)) / refF - 1) < 1e-11
    assert abs(_log_trapezoid(lambda x: G(x) * x ** (mu - 1)) / refG - 1) < 1e-11


def test_small_x_asymptotics(orc):
    a = 4 * math.pi / (math.sqrt(3) * math.gamma(1 / 3)) * 2 ** (-1 / 3)   # 2 M(0) = 2.1495...
    assert abs(a - 2.1495282415) < 1e-9
    for x in (1e-10, 1e-8):
        F, G = orc.synchrotron([x])
        # next terms are O(x^{5/3})
        assert abs(F[0] - (a * x ** (1 / 3) - math.pi / math.sqrt(3) * x)) < 10 * x ** (5 / 3)
        assert abs(G[0] - a / 2 * x ** (1 / 3)) < 10 * x ** (5 / 3)


def test_large_x_asymptotics(orc):
    for x in (100.0, 300.0, 600.0):
        F, G = orc.synchrotron([x])
        lead = math.sqrt(math.pi * x / 2) * math.exp(-x)
        # K_nu asymptotic series (DLMF 10.40.2) for nu = 2/3, two correction terms
        g_ref = lead * (1 + 7 / (72 * x) - 455 / (10368 * x * x))
        assert abs(G[0] / g_ref - 1) < 2.0 / x ** 3
        assert abs(F[0] / (lead * (1 + 55 / (72 * x))) - 1) < 2.0 / x ** 2


def test_printed_values_and_maxima(orc):
    # textbook synchrotron-spectrum maximum F(0.2858) = 0.91801
    xs = np.linspace(0.27, 0.30, 3001)
    F, _ = orc.synchrotron(xs)
    assert abs(xs[np.argmax(F)] - 0.2858) < 2e-4
    assert abs(F.max() - 0.918012) < 2e-6
    xs = np.linspace(0.40, 0.43, 3001)
    _, G = orc.synchrotron(xs)
    assert abs(xs[np.argmax(G)] - 0.4169) < 2e-4
    assert abs(G.max() - 0.607047) < 2e-6


def test_edge_values(orc):
    F, G = orc.synchrotron([0.0, np.inf, 800.0, -1.0, np.nan])
    assert F[0] == 0 and G[0] == 0 and F[1] == 0 and G[1] == 0
    assert F[2] == 0 and G[2] == 0          # underflow
    assert np.isnan(F[3]) and np.isnan(G[3]) and np.isnan(F[4])
