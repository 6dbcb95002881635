"""Pins of the oracle's rates (eqs. (1), (2)), totals, bounds (Sec. 3.1.1), quantum
parameter and pusher, against independent forms: the paper's own double-integral
form of the emission probability, the Baier-Katkov pair spectrum, classical and
asymptotic limits, and textbook identities."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from bessel_ref import int_K

ALPHA = 7.2973525693e-3


@pytest.mark.parametrize("x", [0.05, 0.3, 0.6, 0.9, 0.99])
@pytest.mark.parametrize("chi,gamma", [(0.01, 100.0), (1.0, 1e3), (30.0, 1e4)])
def test_pm_equals_double_integral_form(orc, x, chi, gamma):
    """Sec. 3.1.1: 3x^2 P(x^3) = c x^2 (int_z^inf K_{5/3} + x^6/(1-x^3) K_{2/3}(z)),
    z = x^3/(b(1-x^3)), b = 3 chi/2, c = sqrt(3) alpha dt/(pi gamma)."""
    dt = 123.0
    b = 1.5 * chi
    c = math.sqrt(3) * ALPHA * dt / (math.pi * gamma)
    z = x ** 3 / (b * (1 - x ** 3))
    ref = c * x * x * (int_K(5.0 / 3.0, z) + x ** 6 / (1 - x ** 3) * special.kv(2.0 / 3.0, z))
    got = orc.pm(x, chi, gamma, dt)
    if ref < 1e-290:            # both underflow (z beyond ~700)
        assert got < 1e-290
        return
    assert abs(got / ref - 1) < 1e-11, (got, ref)


@pytest.mark.parametrize("chi_g", [0.5, 2.0, 20.0])
@pytest.mark.parametrize("d", [0.02, 0.2, 0.5, 0.77])
def test_pair_density_equals_baier_katkov(orc, chi_g, d):
    """Eq. (2) with the bracket order corrected equals
    alpha dt /(sqrt(3) pi eps) [(d^2+(1-d)^2)/(d(1-d)) K_{2/3}(xi) + int_xi^inf K_{1/3}],
    xi = 2/(3 chi_g d (1-d))."""
    eps, dt = 50.0, 10.0
    xi = 2.0 / (3.0 * chi_g * d * (1 - d))
    ref = ALPHA * dt / (math.sqrt(3) * math.pi * eps) * (
        (d * d + (1 - d) ** 2) / (d * (1 - d)) * special.kv(2.0 / 3.0, xi) + int_K(1.0 / 3.0, xi))
    got = orc.pp(d, chi_g, eps, dt)
    assert abs(got / ref - 1) < 1e-11, (got, ref)


def test_printed_pair_bracket_is_negative(orc):
    """The bracket as printed, F(z_p) - 3/2 chi_g z_p G(z_p), is negative everywhere."""
    for chi_g in (0.1, 1.0, 10.0, 100.0):
        d = np.linspace(0.01, 0.99, 99)
        zp = 2.0 / (3.0 * chi_g * d * (1 - d))
        F, G = orc.synchrotron(zp)
        printed = F - 1.5 * chi_g * zp * G
        assert np.all(printed[F > 0] < 0)


def test_emission_total_small_chi(orc):
    """Classical limit: total emission rate (5/(2 sqrt 3)) alpha chi / gamma."""
    gamma, dt = 1e3, 1.0
    for chi in (1e-7, 1e-6):
        W = orc.emission_prob(chi, gamma, dt) / dt
        ref = 5.0 / (2.0 * math.sqrt(3.0)) * ALPHA * chi / gamma
        assert abs(W / ref - 1) < 20 * chi


def test_emission_total_large_chi(orc):
    """Quantum limit: W -> 14 Gamma(2/3)/3^{7/3} alpha chi^{2/3} / gamma (slow approach)."""
    gamma, dt, chi = 1e6, 1.0, 1e4
    W = orc.emission_prob(chi, gamma, dt) / dt
    ref = 14.0 * math.gamma(2.0 / 3.0) / 3.0 ** (7.0 / 3.0) * ALPHA * chi ** (2.0 / 3.0) / gamma
    assert 0.99 < W / ref < 1.0


def test_radiated_power_classical_limit(orc):
    """gamma int delta P(delta) d delta / dt = (2/3) alpha chi^2 (1 - 55 sqrt(3)/16 chi + O(chi^2))."""
    gamma, dt = 1e3, 1.0
    for chi in (1e-5, 1e-4):
        P = gamma * orc.emission_energy(chi, gamma, dt) / dt
        ratio = P / (2.0 / 3.0 * ALPHA * chi * chi)
        assert abs(ratio - (1 - 55 * math.sqrt(3) / 16 * chi)) < 60 * chi * chi


def test_pair_total_small_chi(orc):
    """Pair rate at small chi_g: (3 sqrt 3/(16 sqrt 2)) alpha chi_g e^{-8/(3 chi_g)} / eps."""
    eps, dt = 100.0, 1.0
    prev = None
    for chi in (0.02, 0.01, 0.005):
        W = orc.pair_prob(chi, eps, dt) / dt
        ref = 3 * math.sqrt(3) / (16 * math.sqrt(2)) * ALPHA * chi * math.exp(-8 / (3 * chi)) / eps
        err = abs(W / ref - 1)
        assert err < 0.5 * chi
        if prev is not None:
            assert err < prev
        prev = err


@pytest.mark.parametrize("chi_g", [0.7, 8.0])
def test_pair_cdf_against_baier_katkov_quadrature(orc, chi_g):
    """The energy-split CDF of pair creation equals the normalised integral of the
    Baier-Katkov spectrum, by SciPy quadrature of Bessel functions (no oracle code)."""
    def bk(d):
        xi = 2.0 / (3.0 * chi_g * d * (1 - d))
        return (d * d + (1 - d) ** 2) / (d * (1 - d)) * special.kv(2.0 / 3.0, xi) + int_K(1.0 / 3.0, xi)
    tot = 2 * integrate.quad(bk, 1e-12, 0.5, epsrel=1e-11, limit=200)[0]
    for x in (0.05, 0.2, 0.41, 0.5):
        ref = integrate.quad(bk, 1e-12, x, epsrel=1e-11, limit=200)[0] / tot
        assert abs(orc.pair_cdf(chi_g, x) - ref) < 1e-9, (x, orc.pair_cdf(chi_g, x), ref)


def test_pair_cdf_symmetric_and_gaussian_at_small_chi(orc):
    """The split is symmetric, C(x) + C(1 - x) = 1; at small chi_g it is Gaussian around 1/2
    with variance 3 chi_g / 64 (Laplace's method on e^{-z}, z = 2/(3 chi_g x (1 - x)))."""
    for chi in (0.3, 3.0, 40.0):
        for x in (0.03, 0.25, 0.45):
            assert abs(orc.pair_cdf(chi, x) + orc.pair_cdf(chi, 1 - x) - 1) < 1e-12
        assert abs(orc.pair_cdf(chi, 0.5) - 0.5) < 1e-12
    chi = 0.004
    sig = math.sqrt(3 * chi / 64)
    for k in (0.5, 1.0, 2.0):
        phi = 0.5 * (1 + math.erf(k / math.sqrt(2)))
        assert abs(orc.pair_cdf(chi, 0.5 + k * sig) - phi) < 0.02, (k, orc.pair_cdf(chi, 0.5 + k * sig), phi)


def test_emission_bound_is_upper_bound(orc):
    """f(b) of Sec. 3.1.1 exceeds the exact per-step probability for b in [1e-4, 1e3]."""
    gamma, dt = 1e4, 1.0
    ratios = []
    for b in np.logspace(-4, 3, 36):
        chi = b / 1.5
        exact = orc.emission_prob(chi, gamma, dt)
        ratios.append(orc.bound_emission(chi, gamma, dt) / exact)
    ratios = np.array(ratios)
    assert ratios.min() > 1.0 and ratios.max() < 1.4


def test_emission_small_b_constant(orc):
    """As b -> 0 the exact probability tends to (5 pi / 9) c b, which 0.56 pi rounds up."""
    gamma, dt = 1e4, 1.0
    b = 1e-7
    c = math.sqrt(3) * ALPHA * dt / (math.pi * gamma)
    exact = orc.emission_prob(b / 1.5, gamma, dt)
    assert abs(exact / (math.pi * c * b) - 5.0 / 9.0) < 1e-5
    assert abs(orc.bound_emission(b / 1.5, gamma, dt) / (c * b) - (0.56 * math.pi + 0.1)) < 1e-12


def test_emission_bound_pieces(orc):
    """Piece boundaries: each printed breakpoint belongs to the piece above it."""
    gamma, dt = 1.0, 1.0
    c = math.sqrt(3) * ALPHA * dt / (math.pi * gamma)
    for b, coef, p in ((0.05, 0.56, 1.0), (0.1, 0.45, 11 / 12), (0.5, 0.42, 19 / 24),
                       (9.99, 0.42, 19 / 24), (10.0, 0.55, 2 / 3), (500.0, 0.55, 2 / 3)):
        ref = coef * math.pi * c * b ** p + 0.1 * c * b
        assert abs(orc.bound_emission(b / 1.5, gamma, dt) / ref - 1) < 1e-14


def test_pair_bound_violation_window(orc):
    """With c_g = sqrt(3) alpha dt/(pi eps) and b = 3 chi_g/2, 0.1 c b falls below the
    exact pair probability for chi_g between about 3.6 and 69 (it is kept as printed)."""
    eps, dt = 1e3, 1.0
    r = lambda chi: orc.bound_pair(chi, eps, dt, 0.1) / orc.pair_prob(chi, eps, dt)
    assert r(1.0) > 1.0 and r(2.0) > 1.0 and r(100.0) > 1.0
    assert r(5.0) < 1.0 and r(11.4) < 0.8 and r(50.0) < 1.0


def test_nsub_rule(orc):
    assert orc.nsub(0.0, 0.01) == 1
    assert orc.nsub(0.005, 0.01) == 1
    assert orc.nsub(0.03, 0.01) == 3
    assert orc.nsub(0.0301, 0.01) == 4
    assert orc.nsub(1e9, 0.01, 1000) == 1000


def test_chi_identities(orc):
    u = np.array([3.0, -4.0, 12.0])
    g = math.sqrt(1 + u @ u)
    B = np.array([0.0, 0.0, 2e-3])
    zero = np.zeros(3)
    # pure B: chi = |u x B|
    assert abs(orc.chi_lepton(u, zero, B) / np.linalg.norm(np.cross(u, B)) - 1) < 1e-14
    # pure E: chi = |E| sqrt(1 + |u x E|^2/|E|^2)  (Lagrange identity)
    E = np.array([1e-3, 2e-3, -5e-4])
    ref = math.sqrt(E @ E + np.cross(u, E) @ np.cross(u, E))
    assert abs(orc.chi_lepton(u, E, zero) / ref - 1) < 1e-13
    # crossed fields |E| = |B|, E along x, B along y, u along z: chi = |E| (gamma - u_z)
    uz = 50.0
    gz = math.sqrt(1 + uz * uz)
    chi = orc.chi_lepton([0, 0, uz], [1e-3, 0, 0], [0, 1e-3, 0])
    assert abs(chi / (1e-3 / (gz + uz)) - 1) < 1e-9
    # photon: chi_g = eps |B| sin(theta)
    k = np.array([0.0, 600.0, 800.0])
    assert abs(orc.chi_photon(k, zero, np.array([1e-3, 0, 0])) - 1000.0 * 1e-3) < 1e-15
    assert abs(orc.chi_photon(k, zero, np.array([0, 0, 1e-3])) - 1000.0 * 1e-3 * 0.6) < 1e-15


def test_boris_rotation_and_acceleration(orc):
    # pure B: rotation about B by 2 atan(q B dt / (2 gamma)), |u| conserved
    u0 = np.array([30.0, 40.0, 5.0])
    g = math.sqrt(1 + u0 @ u0)
    Bz, dt, q = 2e-2, 7.0, -1.0
    u1 = orc.boris(u0, np.zeros(3), np.array([0, 0, Bz]), q, dt)
    ang = 2 * math.atan(q * Bz * dt / (2 * g))
    rot = np.array([u0[0] * math.cos(ang) + u0[1] * math.sin(ang),
                    -u0[0] * math.sin(ang) + u0[1] * math.cos(ang), u0[2]])
    assert np.allclose(u1, rot, rtol=0, atol=1e-12)
    assert abs(np.linalg.norm(u1) - np.linalg.norm(u0)) < 1e-12
    # pure E: u += q E dt exactly
    E = np.array([1e-3, -2e-3, 4e-3])
    u2 = orc.boris(u0, E, np.zeros(3), +1.0, dt)
    assert np.allclose(u2, u0 + E * dt, rtol=0, atol=1e-13)
