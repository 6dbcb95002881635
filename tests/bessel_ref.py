"""Library-based Bessel integrals used as independent references by the tests."""
import math

from scipy import integrate, special


def int_K(nu, z):
    """int_z^inf K_nu(s) ds with SciPy's K_nu (substitution s = z e^v)."""
    f = lambda v: special.kve(nu, z * math.exp(v)) * math.exp(z - z * math.exp(v)) * z * math.exp(v)
    top = math.log1p(90.0 / z)       # beyond s = z + 90 the tail is below 1e-39 relative
    val, _ = integrate.quad(f, 0, top, epsabs=0, epsrel=1e-13, limit=400)
    return val * math.exp(-z)
