"""The GPU skips the sampling loop of a photon when an upper bound of its pair
density P_p is below the smallest uniform y.  The bound rests on two properties of
G(z) = z K_{2/3}(z), checked here with the oracle: G decreases for z > 0.42, and
G(z) <= sqrt(pi z / 2) e^-z (1 + 7/(72 z)) for z >= 1."""
import math

import numpy as np


def test_G_decreasing_beyond_maximum(orc):
    z = np.linspace(0.42, 50.0, 20000)
    _, G = orc.synchrotron(z)
    assert np.all(np.diff(G) < 0)


def test_G_upper_bound(orc):
    z = np.concatenate([np.linspace(1.0, 10.0, 2000), np.linspace(10.0, 700.0, 2000)])
    _, G = orc.synchrotron(z)
    ub = np.sqrt(np.pi * z / 2) * np.exp(-z) * (1 + 7 / (72 * z))
    ok = G > 0
    assert np.all(G[ok] <= ub[ok] * (1 + 1e-13))


def test_bound_dominates_pair_density(orc):
    """max_x P_p(x) <= A G(8/(3 chi)) for chi where the skip can apply."""
    eps, dt = 300.0, 50.0
    alpha = 7.2973525693e-3
    for chi in (0.05, 0.1, 0.2, 0.5, 2.0):
        x = np.linspace(1e-4, 1 - 1e-4, 4001)
        pmax = max(orc.pp(v, chi, eps, dt) for v in x)
        z0 = (8.0 / 3.0) / chi
        A = alpha * dt * math.sqrt(3) / (2 * math.pi) * chi / eps
        _, G0 = orc.synchrotron([z0])
        assert pmax <= A * G0[0] * (1 + 1e-12)


def test_float_log_domain_test_is_conservative():
    """The kernel evaluates the skip test in float, in the log domain, with a margin of
    1e-3 against ln y_min.  Emulated in numpy float32 over six decades of chi, eps and
    sub-step length: whenever it skips, the bound in double is below y_min; and it
    skips nearly every photon the double test skips."""
    rng = np.random.default_rng(0)
    n = 400000
    chi = 10.0 ** rng.uniform(-3.0, 2.0, n)
    eps = 10.0 ** rng.uniform(0.5, 6.0, n)
    st = 10.0 ** rng.uniform(-2.0, 6.0, n)
    alpha = 7.2973525693e-3
    c = alpha * math.sqrt(3) / (2 * math.pi)
    z0 = (8.0 / 3.0) / chi
    A = c * st * chi / eps
    with np.errstate(over="ignore", under="ignore", invalid="ignore", divide="ignore"):
        ub = 2 * A * np.sqrt(np.pi * z0 / 2) * np.exp(-z0) * (1 + 7 / (72 * z0))
        f = np.float32
        z0f = f(8.0 / 3.0) / chi.astype(f)
        Af = f(c) * st.astype(f) * chi.astype(f) / eps.astype(f)
        lub = np.log(f(2) * Af * np.sqrt(f(0.5 * math.pi) * z0f) * (f(1) + f(7.0 / 72.0) / z0f)) - z0f
    for ymin in (2.0 ** -24, 2.0 ** -53):
        quiet_f = (z0f >= f(1.001)) & (lub < f(math.log(ymin)) - f(1e-3))
        quiet_d = (z0 >= 1.0) & (ub < ymin)
        assert not np.any(quiet_f & ~quiet_d)
        assert np.sum(quiet_f) >= 0.999 * np.sum(quiet_d) and np.sum(quiet_d) > 1000
