"""The pair envelope shipped for the kernels bounds eq. (2) everywhere it is used.

Algorithm 2's exact squeeze in the photon kernel rejects a candidate without
evaluating F and G when its test value y lies above A env(chi) / (3/2 chi), and the
optical-depth path draws the energy split by rejection against env(chi).  Both are
exact only if env(chi) >= D(d) = (3/2) chi (G(z) - d(1-d) F(z)), z = 2/(3 chi d(1-d))
(eq. (2) with its bracket sign-fixed and the factor alpha st sqrt(3)/(2 pi) chi/eps
divided out) for every d, at every chi the kernels can see.  This host test evaluates
the shipped table the way the kernel does (float32: env_j sqrt(chi (1 + chi))
2^(-3.8471867/chi), j = floor(log2 chi) - L0, with a few ulps taken off for the
hardware's approximate sqrt, exp2 and reciprocal, and the neighbouring segment
taken where log2 chi sits next to a segment edge) on 64 chi per octave over the
table's whole range [2^-6, 2^24], against the oracle's F and G at the maximum over d
(a dense grid in d(1-d), refined by a bounded scalar search)."""
import math
import os
import re

import numpy as np
from scipy.optimize import minimize_scalar

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "paper_2008_10468_amd", "csrc", "pair_coeffs.inc")


def _table():
    src = open(INC).read()
    l0 = int(re.search(r"#define QED_PAIR_L0 (-?\d+)", src).group(1))
    nseg = int(re.search(r"#define QED_PAIR_NSEG (\d+)", src).group(1))
    body = re.search(r"qed_pair_env\[\d+\] = \{(.*?)\};", src, re.S).group(1)
    env = np.array([float(v.rstrip("f")) for v in re.findall(r"[-+0-9.eE]+f", body)], np.float32)
    assert env.size == nseg
    return l0, nseg, env


def _envelope_kernel_f32(chi, l0, env, shrink=8):
    """The kernel's env(chi) in float32, lowered by `shrink` ulps of float, the smaller of
    the two segments when log2 chi is within 1e-5 of a segment edge."""
    c = np.float32(chi)
    nseg = env.size
    l = np.log2(np.float64(c))
    segs = {min(max(int(math.floor(l)) - l0, 0), nseg - 1)}
    if abs(l - round(l)) < 1e-5:
        segs.add(min(max(int(round(l)) - l0 - 1, 0), nseg - 1))
        segs.add(min(max(int(round(l)) - l0, 0), nseg - 1))
    root = np.sqrt(np.float32(c * (np.float32(1) + c)), dtype=np.float32)
    e = np.float32(np.exp2(np.float32(-3.8471867) * np.float32(1.0 / np.float64(c))))
    v = min(float(np.float32(env[j] * root * e)) for j in segs)
    if v < 2.0 ** -126:      # results below the normal range may be flushed to zero
        return 0.0
    return v * (1.0 - shrink * 2.0 ** -24)


def _density_max(orc, chi):
    """max over d of (3/2) chi (G(z) - u F(z)), u = d (1 - d) in (0, 1/4], z = 2 / (3 chi u)."""
    def dens(u):
        z = 2.0 / (3.0 * chi * u)
        F, G = orc.synchrotron(np.atleast_1d(z))
        return 1.5 * chi * (G - u * F)
    lu = np.linspace(math.log(1e-9), math.log(0.25), 400)
    v = dens(np.exp(lu))
    k = int(np.argmax(v))
    lo, hi = lu[max(k - 1, 0)], lu[min(k + 1, lu.size - 1)]
    r = minimize_scalar(lambda t: -float(dens(np.exp([t]))[0]), bounds=(lo, hi), method="bounded",
                        options={"xatol": 1e-10})
    return max(float(v.max()), -float(r.fun))


# A = alpha st sqrt(3)/(2 pi) chi/eps, the factor between D / (3/2 chi) and P_p, stays far
# below this for any sub-step a QED-PIC code takes (chi/eps is the field across the
# photon, at most a few Schwinger units, and alpha st < 1e6 for st < 1e8 hbar/mc^2).
A_MAX = 1e6
Y_MIN = 2.0 ** -53          # the smallest test value y either path draws


def test_envelope_bounds_the_pair_density(orc):
    """env(chi) >= D(d) with 1e-5 to spare (the kernels' F and G are fits good to 2e-6),
    except where the float envelope underflows (chi below about 0.026): there D is
    so small that A_MAX D / (3/2 chi) < 2^-53, so no test value can fall below P_p and
    rejecting every candidate is the decision eq. (2) gives."""
    l0, nseg, env = _table()
    chis = 2.0 ** (l0 + np.arange(nseg * 64 + 1) / 64.0)
    worst, where, quiet = np.inf, None, 0
    for chi in chis:
        dmax = _density_max(orc, chi)
        e = _envelope_kernel_f32(chi, l0, env)
        if e < dmax * (1.0 + 1e-5):
            assert A_MAX * dmax / (1.5 * chi) < Y_MIN, (chi, e, dmax)
            quiet += 1
            continue
        if e / dmax < worst:
            worst, where = e / dmax, chi
    assert worst >= 1.0 + 1e-5, (worst, where)
    assert quiet < 64, quiet     # only the bottom of the table (chi < 2^-5.2) is below the envelope


def test_envelope_is_not_loose(orc):
    """The margin is what the fit intends (5% above the sampled maxima), not a
    bound so loose that the squeeze and the rejection sampler lose their use."""
    l0, nseg, env = _table()
    chis = 2.0 ** (l0 + 2 + np.arange((nseg - 2) * 8 + 1) / 8.0)
    ratios = [_envelope_kernel_f32(chi, l0, env, shrink=0) / _density_max(orc, chi) for chi in chis]
    assert max(ratios) < 1.35, max(ratios)


# ---------------------------------------------------------------------------
# The emission envelope of the optical-depth path's rejection sampler: on segment j
# of log2 chi, ((1 - x^3) F(z) + x^6 G(z)) / x <= env_j b^(-1/3) for every x in (0, 1),
# z = x^3 / (b (1 - x^3)), b = 3 chi / 2 (eq. (1) over c b); a constant above the table.
# A candidate above the envelope is counted (envelope_clips) rather than lost, but a
# bound that holds keeps the sampler exact.
# ---------------------------------------------------------------------------
RATE_INC = os.path.join(ROOT, "paper_2008_10468_amd", "csrc", "rate_coeffs.inc")


def _rate_table():
    src = open(RATE_INC).read()
    l0 = int(re.search(r"#define QED_RATE_L0 (-?\d+)", src).group(1))
    nseg = int(re.search(r"#define QED_RATE_NSEG (\d+)", src).group(1))
    top = float(re.search(r"#define QED_RATE_ENV_TOP ([-+0-9.eE]+)f", src).group(1))
    body = re.search(r"qed_rate_env\[\d+\] = \{(.*?)\};", src, re.S).group(1)
    env = np.array([float(v.rstrip("f")) for v in re.findall(r"[-+0-9.eE]+f", body)], np.float32)
    assert env.size == nseg
    return l0, nseg, top, env


def _rate_envelope_f32(chi, l0, nseg, top, env, shrink=8):
    c = np.float32(chi)
    l = np.log2(np.float64(c))
    if l >= l0 + nseg:
        return top * (1.0 - shrink * 2.0 ** -24)
    segs = {min(max(int(math.floor(l)) - l0, 0), nseg - 1)}
    if abs(l - round(l)) < 1e-5:
        segs.add(min(max(int(round(l)) - l0 - 1, 0), nseg - 1))
        segs.add(min(max(int(round(l)) - l0, 0), nseg - 1))
    bm13 = np.float32(np.exp2(-(np.float32(l) + np.float32(0.58496250072)) * np.float32(1.0 / 3.0)))
    return min(float(np.float32(env[j] * bm13)) for j in segs) * (1.0 - shrink * 2.0 ** -24)


def _emission_density_max(orc, chi):
    """max over x in (0, 1) of ((1 - x^3) F(z) + x^6 G(z)) / x, z = x^3 / (b (1 - x^3))."""
    b = 1.5 * chi

    def dens(x):
        x3 = x ** 3
        om = (1.0 - x) * (1.0 + x + x * x)
        F, G = orc.synchrotron(x3 / (b * om))
        return (om * F + x3 * x3 * G) / x
    lx = np.linspace(math.log(1e-12), math.log(1.0 - 1e-9), 600)
    v = dens(np.exp(lx))
    k = int(np.argmax(v))
    lo, hi = lx[max(k - 1, 0)], lx[min(k + 1, lx.size - 1)]
    r = minimize_scalar(lambda t: -float(dens(np.exp([t]))[0]), bounds=(lo, hi), method="bounded",
                        options={"xatol": 1e-12})
    return max(float(v.max()), -float(r.fun))


def test_emission_envelope_bounds_eq1(orc):
    """16 chi per octave over the table [2^-30, 2^16] and four octaves above it."""
    l0, nseg, top, env = _rate_table()
    chis = 2.0 ** (l0 + np.arange((nseg + 4) * 16 + 1) / 16.0)
    worst, where = np.inf, None
    for chi in chis:
        r = _rate_envelope_f32(chi, l0, nseg, top, env) / _emission_density_max(orc, chi)
        if r < worst:
            worst, where = r, chi
    assert worst >= 1.0 + 1e-5, (worst, where)
