"""Pins of the oracle's Algorithms 1 and 2: brute force on tiny cases, exact
distributions in a uniform magnetic field (where Boris keeps gamma and chi fixed
between events), conservation laws and determinism."""
import math

import numpy as np
import pytest
from scipy import special

from bessel_ref import int_K

ALPHA = 7.2973525693e-3


def _species(n, u, id0=0):
    s = {k: np.zeros(n) for k in ("x", "y", "z")}
    s["ux"] = np.full(n, float(u[0]))
    s["uy"] = np.full(n, float(u[1]))
    s["uz"] = np.full(n, float(u[2]))
    s["w"] = np.linspace(0.5, 2.0, n)
    s["id"] = np.arange(id0, id0 + n, dtype=np.uint64)
    return s


def _field(E=(0, 0, 0), B=(0, 0, 0)):
    return {k: np.array([float(v)]) for k, v in zip(("ex", "ey", "ez", "bx", "by", "bz"), tuple(E) + tuple(B))}


def _pm_by_hand(x, chi, gamma, dt):
    """3x^2 P(x^3) from the double-integral form of Sec. 3.1.1 with SciPy Bessel functions."""
    b = 1.5 * chi
    c = math.sqrt(3) * ALPHA * dt / (math.pi * gamma)
    z = x ** 3 / (b * (1 - x ** 3))
    if z > 700:
        return 0.0
    return c * x * x * (int_K(5 / 3, z) + x ** 6 / (1 - x ** 3) * special.kv(2 / 3, z))


@pytest.mark.parametrize("rng_bits", [53, 24])
def test_single_substep_brute_force(orc, rng_bits):
    """Particles with N = 1: every accept decision, photon and recoil recomputed by hand."""
    gamma = 2000.0
    u = math.sqrt(gamma * gamma - 1)
    Bz = 2.0e-4                    # chi = 0.4 for u perpendicular to B
    chi = u * Bz
    dt = 0.0095 / orc.bound_emission(chi, gamma, 1.0)      # f = 0.0095 -> N = 1
    n = 3000
    st = _species(n, (u, 0, 0))
    q0 = {k: v.copy() for k, v in st.items()}
    seed, step = 99, 5
    ch, nsub, nev, tally = orc.lepton_step(st, _field(B=(0, 0, Bz)), -1.0, dt, seed, step,
                                           p_max=0.01, rng_bits=rng_bits)
    assert np.all(nsub == 1)
    f = orc.bound_emission(chi, gamma, dt)
    assert f <= 0.01
    # Boris rotation for one sub-step (pure B keeps |u|)
    ang = 2 * math.atan(-Bz * dt / (2 * gamma))
    dirx, diry = math.cos(ang), -math.sin(ang)
    n_ev = 0
    for i in range(n):
        x, y = orc.draw_xy(seed, int(q0["id"][i]), step, 0, rng_bits)
        pm = _pm_by_hand(x, chi, gamma, dt)
        event = y < pm
        assert bool(nev[i]) == event, (i, x, y, pm)
        if event:
            j = np.flatnonzero(ch["parent"] == q0["id"][i])
            assert j.size == 1
            j = j[0]
            delta = x ** 3
            assert abs(ch["px"][j] - delta * gamma * dirx) < 1e-9 * gamma
            assert abs(ch["py"][j] - delta * gamma * diry) < 1e-9 * gamma
            assert ch["w"][j] == q0["w"][i]
            assert ch["id"][j] == orc.child_id(seed, int(q0["id"][i]), step, 0, 0)
            g1 = (1 - delta) * gamma
            assert abs(math.hypot(st["ux"][i], st["uy"][i]) - math.sqrt(g1 * g1 - 1)) < 1e-9 * gamma
            # energy conservation: gamma = gamma' + eps_photon
            eps = math.hypot(ch["px"][j], ch["py"][j])
            assert abs(math.sqrt(1 + st["ux"][i] ** 2 + st["uy"][i] ** 2) + eps - gamma) < 1e-9 * gamma
            n_ev += 1
    assert n_ev > 5 and ch["id"].size == n_ev
    assert tally["events"] == n_ev and tally["substeps"] == n


def test_uniform_B_first_event_statistics(orc):
    """In a uniform B field gamma and chi stay fixed until the first event, so the
    number of event-free steps is Binomial(n, (1-p)^N) and the sub-step index of the
    first event is geometric, with p = int_0^1 min(P_m, 1) dx per sub-step."""
    gamma = 1000.0
    u = math.sqrt(gamma * gamma - 1)
    Bz = 1e-3
    chi = u * Bz
    dt = 3.0e4
    n = 6000
    st = _species(n, (u, 0, 0))
    ch, nsub, nev, tally = orc.lepton_step(st, _field(B=(0, 0, Bz)), -1.0, dt, 3, 0)
    N = int(nsub[0])
    assert np.all(nsub == N) and 5 < N < 200
    p = orc.emission_prob(chi, gamma, dt / N, clip=True)
    p0 = (1 - p) ** N
    k0 = int(np.sum(nev == 0))
    assert abs(k0 - n * p0) < 4 * math.sqrt(n * p0 * (1 - p0))
    # first-event sub-step index: geometric truncated at N
    first = {}
    for par, sub in zip(ch["parent"], ch["sub"]):
        first[int(par)] = min(first.get(int(par), N), int(sub))
    idx = np.array(list(first.values()))
    probs = np.array([(1 - p) ** i * p for i in range(N)]) / (1 - p0)
    nb = 8
    edges = np.linspace(0, N, nb + 1).astype(int)
    obs = np.array([np.sum((idx >= edges[j]) & (idx < edges[j + 1])) for j in range(nb)])
    exp = np.array([probs[edges[j]:edges[j + 1]].sum() for j in range(nb)]) * idx.size
    chi2 = float(np.sum((obs - exp) ** 2 / exp))
    assert chi2 < 24          # 7 dof, p ~ 1e-3


def test_uniform_B_first_event_spectrum(orc):
    """The photon energy fraction of first events follows the normalised spectrum of
    eq. (1): CDF C(delta) = int_0^{delta^(1/3)} P_m / int_0^1 P_m (KS test)."""
    gamma = 1000.0
    u = math.sqrt(gamma * gamma - 1)
    Bz = 2e-3
    chi = u * Bz
    dt = 2.0e4
    n = 5000
    st = _species(n, (u, 0, 0))
    ch, nsub, nev, tally = orc.lepton_step(st, _field(B=(0, 0, Bz)), -1.0, dt, 11, 2)
    first = {}
    for j, (par, sub) in enumerate(zip(ch["parent"], ch["sub"])):
        if int(par) not in first or sub < ch["sub"][first[int(par)]]:
            first[int(par)] = j
    js = np.array(sorted(first.values()))
    delta = np.hypot(ch["px"][js], ch["py"][js]) / gamma
    delta.sort()
    grid = np.quantile(delta, np.linspace(0.02, 0.98, 25))
    cdf = np.array([orc.emission_cdf(chi, d) for d in grid])
    emp = np.searchsorted(delta, grid, side="right") / delta.size
    assert np.max(np.abs(cdf - emp)) < 1.63 / math.sqrt(delta.size)


def test_photon_survival_and_pair_sharing(orc):
    """A photon in a uniform B survives a step with probability (1 - p_p)^N; the pair
    shares its energy: gamma_e + gamma_p = eps (above threshold)."""
    eps = 2000.0
    Bz = 2e-3
    chi = eps * Bz           # k along x, B along z
    dt = 3.0e4
    n = 6000
    st = _species(n, (eps, 0, 0), id0=10 ** 6)
    ch, alive, nsub, nev, tally = orc.photon_step(st, _field(B=(0, 0, Bz)), dt, 5, 1)
    N = int(nsub.max())
    assert N > 3
    pp = orc.pair_prob(chi, eps, dt / N, clip=True)
    ps = (1 - pp) ** N
    k = int(alive.sum())
    assert abs(k - n * ps) < 4 * math.sqrt(n * ps * (1 - ps))
    e = ch["kind"] == 1
    p = ch["kind"] == 2
    assert e.sum() == p.sum() == n - k
    ge = np.sqrt(1 + ch["px"][e] ** 2)
    gp = np.sqrt(1 + ch["px"][p] ** 2)
    assert np.allclose(ge + gp, eps, rtol=1e-12)
    assert np.array_equal(ch["parent"][e], ch["parent"][p])
    # positions advanced at the speed of light to the decay sub-step
    for j in np.flatnonzero(e)[:50]:
        assert abs(ch["x"][j] - (ch["sub"][j] + 1) * dt / N) < 1e-9 * dt


def test_chunking_and_threads_do_not_change_results(orc):
    import workloads
    w = workloads.c1(n=1500)
    outs = []
    for threads in (1, 8):
        st = {k: v.copy() for k, v in w["electrons"].items()}
        ch, nsub, nev, tally = orc.lepton_step(st, w["fields"], -1.0, w["dt"], 1, 0, threads=threads)
        outs.append((st, ch, nsub, nev))
    for k in ("ux", "uy", "uz", "x", "y", "z"):
        assert np.array_equal(outs[0][0][k], outs[1][0][k])
    for k in ("id", "px", "parent", "sub"):
        assert np.array_equal(outs[0][1][k], outs[1][1][k])
    assert np.array_equal(outs[0][3], outs[1][3])


def test_degenerate_inputs(orc):
    st = _species(4, (100.0, 0, 0))
    st["uy"][1] = np.nan
    st["ux"][2] = 0.0          # at rest
    ch, nsub, nev, tally = orc.lepton_step(st, _field(), -1.0, 1e4, 1, 0)
    # zero field: chi = 0, one sub-step, no event, particle moves ballistically
    assert tally["nonfinite"] == 1 and nsub[1] == 0 and np.isnan(st["uy"][1])
    assert list(nsub[[0, 2, 3]]) == [1, 1, 1] and nev.sum() == 0 and ch["id"].size == 0
    assert st["x"][2] == 0.0 and abs(st["x"][0] - 1e4 * 100 / math.sqrt(1 + 1e4)) < 1e-6
    ph = _species(2, (0.0, 0, 0), id0=50)
    ch, alive, nsub, nev, tally = orc.photon_step(ph, _field(B=(0, 0, 1)), 1e4, 1, 0)
    assert np.all(alive == 1) and np.all(nsub == 1) and ch["id"].size == 0
