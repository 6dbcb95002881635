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
