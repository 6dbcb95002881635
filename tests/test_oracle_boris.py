"""Pins of the oracle's push (Algorithms 1 and 2 move every lepton by a Boris step in
the frozen field between candidates) and of its quantum parameter in fields where E
and B are both non-zero and not orthogonal.

Each pin comes from outside the oracle: an exact property of the rotation inside
the Boris step, an independent ODE integration of du/dt = q (E + u x B / gamma)
(second-order convergence of momentum and position), the guiding-centre drift
E x B / B^2 of crossed fields, and chi as the electric field in the particle's rest
frame (a Lorentz boost, not the invariant formula the oracle evaluates).  A dropped
half kick, a half kick of the wrong sign or order, gamma taken before the first half
kick, or a transposed cross product each fails at least one of them."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp


def _rand_dir(rng):
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def _fields(rng, e_mag, b_mag):
    """E and B of the given magnitudes in general (non-orthogonal) directions."""
    return e_mag * _rand_dir(rng), b_mag * _rand_dir(rng)


@pytest.mark.parametrize("seed", range(6))
def test_rotation_keeps_the_norm_between_half_kicks(orc, seed):
    """The magnetic part of the step is a rotation, so with u- = u0 + hE and
    u+ = u1 - hE (h = q dt / 2): |u+| = |u-|, i.e. |u1|^2 - |u0|^2 = q dt E.(u0 + u1).
    A wrong order of kick and rotation breaks this identity."""
    rng = np.random.default_rng(seed)
    u0 = rng.standard_normal(3) * 10.0 ** rng.uniform(0, 3)
    E, B = _fields(rng, 10.0 ** rng.uniform(-4, -2), 10.0 ** rng.uniform(-4, -2))
    q = -1.0 if seed % 2 else 1.0
    dt = 10.0 ** rng.uniform(1, 3)
    u1 = orc.boris(u0, E, B, q, dt)
    lhs = u1 @ u1 - u0 @ u0
    rhs = q * dt * (E @ (u0 + u1))
    scale = max(abs(lhs), 1e-12 * (u1 @ u1 + u0 @ u0))
    assert abs(lhs - rhs) <= 1e-10 * scale, (lhs, rhs)
    # and the rotation is about B: the component of u along B changes only by the kicks
    bh = B / np.linalg.norm(B)
    assert abs((u1 - u0 - q * dt * E) @ bh) <= 1e-10 * max(np.linalg.norm(u0), 1.0)


def _ode_reference(u0, E, B, q, t_end, t_eval):
    """u(t) and x(t) of du/dt = q (E + u x B / gamma), dx/dt = u / gamma by an 8th-order
    Runge-Kutta method at tight tolerances (SciPy; no oracle code)."""
    def rhs(t, y):
        u = y[:3]
        g = math.sqrt(1.0 + u @ u)
        return np.concatenate([q * (E + np.cross(u, B) / g), u / g])
    sol = solve_ivp(rhs, (0.0, t_end), np.concatenate([u0, np.zeros(3)]), method="DOP853",
                    rtol=1e-13, atol=1e-12, t_eval=t_eval, dense_output=True)
    assert sol.success
    return sol


def _push_path(orc, u0, E, B, q, st, n):
    """n oracle Boris steps, the position advanced by each new velocity (the order the
    oracle's Algorithm 1 uses)."""
    u = np.array(u0, np.float64)
    x = np.zeros(3)
    for _ in range(n):
        u = orc.boris(u, E, B, q, st)
        x += u / math.sqrt(1.0 + u @ u) * st
    return u, x


@pytest.mark.parametrize("seed,q", [(0, -1.0), (1, 1.0), (2, -1.0)])
def test_second_order_convergence_in_combined_fields(orc, seed, q):
    """Boris is a time-centred second-order scheme: halving the sub-step divides the
    momentum error at a fixed time by four.  u after n steps approximates the exact
    momentum at t = n st (the velocity is staggered by half a step, and the fields are
    static, so the shift does not matter for u); the position after n steps
    approximates x(t + st/2) - x(st/2) of the exact path."""
    rng = np.random.default_rng(100 + seed)
    E, B = _fields(rng, 4e-4, 1e-3)                    # |E| < |B|, general angle
    u0 = rng.standard_normal(3) * 5.0
    g0 = math.sqrt(1.0 + u0 @ u0)
    T = 2.5 * 2 * math.pi * g0 / 1e-3                  # a few gyration periods
    sol = _ode_reference(u0, E, B, q, T + T / 100, None)
    errs_u, errs_x = [], []
    for n in (400, 800, 1600):
        st = T / n
        u, x = _push_path(orc, u0, E, B, q, st, n)
        ref = sol.sol(T)
        xr = sol.sol(T + st / 2)[3:] - sol.sol(st / 2)[3:]
        errs_u.append(np.linalg.norm(u - ref[:3]) / np.linalg.norm(ref[:3]))
        errs_x.append(np.linalg.norm(x - xr) / np.linalg.norm(xr))
    for errs in (errs_u, errs_x):
        r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
        assert 3.4 < r1 < 4.6 and 3.4 < r2 < 4.6, errs
    assert errs_u[-1] < 1e-3 and errs_x[-1] < 1e-3, (errs_u, errs_x)


def test_exb_drift(orc):
    """Crossed fields, |E| = |B|/2, E perpendicular to B, particle starting at rest: the
    guiding centre drifts at v_d = E x B / B^2 (relativistic, |v_d| = 0.5).  The mean
    velocity over many gyrations approaches v_d."""
    rng = np.random.default_rng(7)
    bh = _rand_dir(rng)
    eh = np.cross(bh, _rand_dir(rng))
    eh /= np.linalg.norm(eh)
    Bm = 1e-3
    E, B = 0.5 * Bm * eh, Bm * bh
    vd = np.cross(E, B) / (B @ B)
    # In the frame moving with v_d the field is B / gamma_d (no E) and the particle
    # gyrates with gamma' = gamma_d, so its period there is 2 pi gamma_d^2 / |B|; the
    # lab period is gamma_d times longer (gamma_d = 1/sqrt(1 - v_d^2)).
    gd = 1.0 / math.sqrt(1.0 - vd @ vd)
    period = 2 * math.pi * gd ** 3 / Bm
    n_per = 400
    st = period / n_per
    u, x = _push_path(orc, np.zeros(3), E, B, -1.0, st, 40 * n_per)
    vmean = x / (40 * period)
    assert np.linalg.norm(vmean - vd) < 2e-3 * np.linalg.norm(vd), (vmean, vd)


def _chi_rest_frame(u, E, B):
    """|E'| in the rest frame of a lepton with momentum u (units of E_S):
    E' = gamma (E + v x B) - gamma^2/(gamma+1) v (v . E)."""
    g = math.sqrt(1.0 + u @ u)
    v = u / g
    Ep = g * (E + np.cross(v, B)) - g * g / (g + 1.0) * v * (v @ E)
    return np.linalg.norm(Ep)


@pytest.mark.parametrize("seed", range(8))
def test_chi_is_the_rest_frame_field(orc, seed):
    """chi of a lepton equals the electric field in its rest frame, for E and B both
    non-zero at a general angle."""
    rng = np.random.default_rng(200 + seed)
    u = _rand_dir(rng) * 10.0 ** rng.uniform(0, 4)
    E, B = _fields(rng, 10.0 ** rng.uniform(-4, -2), 10.0 ** rng.uniform(-4, -2))
    got = orc.chi_lepton(u, E, B)
    ref = _chi_rest_frame(u, E, B)
    assert abs(got / ref - 1) < 1e-9, (got, ref)


def test_oracle_step_moves_like_its_pushes(orc):
    """The oracle's Algorithm 1 with forced sub-steps and no possible emission (chi about
    1e-9) moves each lepton exactly as n single Boris steps plus moves do, in a field
    with E and B both non-zero."""
    rng = np.random.default_rng(11)
    n = 16
    E, B = _fields(rng, 2e-9, 5e-9)
    st_ = {"ux": rng.standard_normal(n) * 3, "uy": rng.standard_normal(n) * 3, "uz": rng.standard_normal(n) * 3,
           "x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n), "w": np.ones(n),
           "id": np.arange(n, dtype=np.uint64)}
    u0 = np.stack([st_["ux"], st_["uy"], st_["uz"]], axis=1).copy()
    fields = {k: np.array([v]) for k, v in zip(("ex", "ey", "ez", "bx", "by", "bz"), (*E, *B))}
    dt, nsub = 3.0e6, 37
    _, ns, nev, _ = orc.lepton_step(st_, fields, -1.0, dt, 1, 0, nsub=np.full(n, nsub, np.uint32))
    assert np.all(ns == nsub) and np.all(nev == 0)
    for i in range(n):
        u, x = _push_path(orc, u0[i], E, B, -1.0, dt / nsub, nsub)
        assert np.allclose([st_["ux"][i], st_["uy"][i], st_["uz"][i]], u, rtol=1e-14, atol=0)
        assert np.allclose([st_["x"][i], st_["y"][i], st_["z"][i]], x, rtol=1e-12, atol=1e-9)
