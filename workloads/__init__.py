"""Seeded synthetic initial conditions for the QED event-generator workloads.

This module is shared by the tests, the benchmark and the oracle runs.  It only
draws random numbers and lays them out; it holds none of the generator's
arithmetic (no rates, no bounds, no quantum parameter).  Each workload mirrors
the regime a QED-PIC push stage sees (Sec. 2.2 and 3.1 of the paper):

* ``c1``  16,384 electrons, gamma log-uniform in [1e2, 1e4], isotropic, uniform
          static B = 1e-3 (Schwinger units) along z; chi spans about [1e-2, 10].
* ``c2``  1,048,576 electrons + 262,144 photons in a uniform E field of amplitude
          1e-3 rotating in the xy plane with period 200 dt; chi and gamma drawn
          jointly (chi log-uniform in [1e-3, 1e2], gamma log-uniform in
          [max(10, 1e3 chi), 1e5], pitch angle to E from sin(theta) = chi/(E gamma)).
* ``c3``  16,777,216 electrons, gamma log-uniform in [1e3, 1e4], isotropic; 90% in
          a weak field B = 5e-7 z (chi < 5e-3, one sub-step), 10% in a Gaussian
          hot spot B = 1e-2 exp(-r^2/2) z with r ~ N(0, I_3) in units of the spot
          size; fields are per particle and static.
* ``c4``  log-uniform x in [1e-4, 50] for the synchrotron-function microbenchmark.
* ``shower``  in-step cascades: electrons, positrons and photons in equal numbers,
          gamma (photon energy) log-uniform in [1e4, 10^5.5], isotropic, uniform
          static B = 2e-3 along z, dt = 3e5: particles created early in the step
          create further particles within it, five to six generations deep.

All species arrays are float64 numpy arrays (``x, y, z, ux, uy, uz, w``) plus
uint64 ``id``; photon momenta are stored in ``ux, uy, uz`` as k = hbar k/(m c).
Ids are unique across species.  Sizes can be scaled down with ``scale`` (tests).
"""
from __future__ import annotations

import math

import numpy as np

# Global steps (units hbar/(m c^2)).  Fixed here; how each value was chosen is
# stated beside it.
DT_C1 = 8.37e4         # mean emission probability per step about 0.5
DT_C2 = 10358.420305623711   # (0.8 um laser period) / 200
DT_C3 = 2.0696e5       # hot-spot particles need at most 1000 sub-steps
DT_SHOWER = 3.0e5      # five to six generations of events inside one step
B_SHOWER = 2.0e-3
E0_C2 = 1.0e-3
B_C1 = 1.0e-3
P_MAX = 0.01


def _isotropic(rng, n):
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return sth * np.cos(phi), sth * np.sin(phi), cth


def _species(n, id0, rng, pos_scale=1.0e4):
    return {
        "x": rng.uniform(-pos_scale, pos_scale, n),
        "y": rng.uniform(-pos_scale, pos_scale, n),
        "z": rng.uniform(-pos_scale, pos_scale, n),
        "w": np.ones(n),
        "id": np.arange(id0, id0 + n, dtype=np.uint64),
    }


def _empty():
    s = {k: np.zeros(0) for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
    s["id"] = np.zeros(0, np.uint64)
    return s


def cell_box(n_per_axis, pos_scale=1.0e4):
    """Cell geometry covering the cube [-pos_scale, pos_scale)^3 in which the workloads
    place their particles, n_per_axis cells along each axis (for sub-steps per cell)."""
    d = 2.0 * pos_scale / n_per_axis
    return {"nx": n_per_axis, "ny": n_per_axis, "nz": n_per_axis, "x0": -pos_scale, "y0": -pos_scale,
            "z0": -pos_scale, "dx": d, "dy": d, "dz": d}


def uniform_field(ex=0.0, ey=0.0, ez=0.0, bx=0.0, by=0.0, bz=0.0):
    return {k: np.array([v], np.float64) for k, v in
            zip(("ex", "ey", "ez", "bx", "by", "bz"), (ex, ey, ez, bx, by, bz))}


def c1(n=16384, seed=1):
    """Emission only, FP64 path: electrons in a uniform static magnetic field."""
    rng = np.random.default_rng(seed)
    e = _species(n, 0, rng)
    gamma = 10.0 ** rng.uniform(2.0, 4.0, n)
    u = np.sqrt(gamma * gamma - 1.0)
    dx, dy, dz = _isotropic(rng, n)
    e["ux"], e["uy"], e["uz"] = u * dx, u * dy, u * dz
    return {"electrons": e, "positrons": _empty(), "photons": _empty(),
            "fields": uniform_field(bz=B_C1), "dt": DT_C1, "steps": 100, "seed": 1,
            "p_max": P_MAX}


def shower(n=4096, seed=6):
    """In-step cascades: n electrons, n positrons and n photons seeding a shower."""
    rng = np.random.default_rng(seed)
    out = {}
    for k, name in enumerate(("electrons", "positrons", "photons")):
        s = _species(n, k * n, rng)
        energy = 10.0 ** rng.uniform(4.0, 5.5, n)
        u = energy if name == "photons" else np.sqrt(energy * energy - 1.0)
        dx, dy, dz = _isotropic(rng, n)
        s["ux"], s["uy"], s["uz"] = u * dx, u * dy, u * dz
        out[name] = s
    out.update({"fields": uniform_field(bz=B_SHOWER), "dt": DT_SHOWER, "steps": 4, "seed": 1,
                "p_max": P_MAX})
    return out


def _joint_chi_energy(rng, n, e0):
    """chi log-uniform in [1e-3, 1e2]; energy log-uniform in [max(10, 1e3 chi), 1e5];
    direction at angle theta to x with sin(theta) = chi / (e0 * energy)."""
    chi = 10.0 ** rng.uniform(-3.0, 2.0, n)
    lo = np.log10(np.maximum(10.0, 1.0e3 * chi))
    energy = 10.0 ** (lo + (5.0 - lo) * rng.uniform(0.0, 1.0, n))
    sth = np.clip(chi / (e0 * energy), 0.0, 1.0)
    cth = np.sqrt(1.0 - sth * sth) * np.where(rng.uniform(0, 1, n) < 0.5, -1.0, 1.0)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    # axis x is the field direction at step 0
    return energy, (cth, sth * np.cos(phi), sth * np.sin(phi))


def c2(n_e=1048576, n_g=262144, seed=2):
    """Emission + pair creation, mixed precision, rotating uniform E field."""
    rng = np.random.default_rng(seed)
    e = _species(n_e, 0, rng)
    gamma, (dx, dy, dz) = _joint_chi_energy(rng, n_e, E0_C2)
    u = np.sqrt(np.maximum(gamma * gamma - 1.0, 0.0))
    e["ux"], e["uy"], e["uz"] = u * dx, u * dy, u * dz
    g = _species(n_g, n_e, rng)
    eps, (dx, dy, dz) = _joint_chi_energy(rng, n_g, E0_C2)
    g["ux"], g["uy"], g["uz"] = eps * dx, eps * dy, eps * dz
    return {"electrons": e, "positrons": _empty(), "photons": g,
            "fields": c2_field(0), "dt": DT_C2, "steps": 200, "seed": 1, "p_max": P_MAX}


def c2_field(step, steps_per_turn=200):
    """E(t) = E0 (cos 2 pi s/200, sin 2 pi s/200, 0), frozen over global step s."""
    ph = 2.0 * math.pi * step / steps_per_turn
    return uniform_field(ex=E0_C2 * math.cos(ph), ey=E0_C2 * math.sin(ph))


def c3(n=16777216, seed=3, hot_fraction=0.1, shuffle=True):
    """Uneven batch: weak-field bulk plus a Gaussian hot spot (per-particle fields)."""
    rng = np.random.default_rng(seed)
    e = _species(n, 0, rng)
    gamma = 10.0 ** rng.uniform(3.0, 4.0, n)
    u = np.sqrt(gamma * gamma - 1.0)
    dx, dy, dz = _isotropic(rng, n)
    e["ux"], e["uy"], e["uz"] = u * dx, u * dy, u * dz
    n_hot = int(round(hot_fraction * n))
    hot = np.zeros(n, bool)
    hot[:n_hot] = True
    if shuffle:
        rng.shuffle(hot)
    r2 = np.sum(rng.standard_normal((3, n)) ** 2, axis=0)
    bz = np.where(hot, 1.0e-2 * np.exp(-0.5 * r2), 5.0e-7)
    zeros = np.zeros(n)
    fields = {"ex": zeros, "ey": zeros, "ez": zeros, "bx": zeros, "by": zeros, "bz": bz}
    return {"electrons": e, "positrons": _empty(), "photons": _empty(), "fields": fields,
            "hot": hot, "dt": DT_C3, "steps": 50, "seed": 1, "p_max": P_MAX}


DT_WEAK = 1.0e8        # weak uniform field: about 0.8 emissions per electron and step
B_WEAK = 1.0e-6


def weak(n=16777216, seed=8):
    """Every electron in one weak uniform field (chi 1e-3 to 1e-2, about 90 sub-steps of
    Algorithm 1 at P_max = 0.01): the emission spectrum is concentrated at small x, where
    the rejection sampler's flat envelope accepts one candidate in five to ten."""
    rng = np.random.default_rng(seed)
    e = _species(n, 0, rng)
    gamma = 10.0 ** rng.uniform(3.0, 4.0, n)
    u = np.sqrt(gamma * gamma - 1.0)
    dx, dy, dz = _isotropic(rng, n)
    e["ux"], e["uy"], e["uz"] = u * dx, u * dy, u * dz
    return {"electrons": e, "positrons": _empty(), "photons": _empty(), "fields": uniform_field(bz=B_WEAK),
            "dt": DT_WEAK, "steps": 20, "seed": 1, "p_max": P_MAX}


def c4_host(n, seed=4):
    """log-uniform x in [1e-4, 50] (host, float64)."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(-4.0, math.log10(50.0), n)


def subset(species, idx):
    return {k: np.ascontiguousarray(v[idx]) for k, v in species.items()}


def field_subset(fields, idx):
    out = {}
    for k, v in fields.items():
        out[k] = v if v.size == 1 else np.ascontiguousarray(v[idx])
    return out


# ---------------------------------------------------------------------------
# General electromagnetic fields (E and B both non-zero, at general angles), as a
# field interpolated from a PIC grid gives them.
# ---------------------------------------------------------------------------
DT_GENERAL = 3.0e4      # mean emission probability per step about 0.3
DT_CROSSED = 1.0e7      # crossed fields near |E| = |B|: the rate is small, the step long


def _field_modes(seed, m=4):
    """Random plane-wave-like modes: amplitude vector, wave vector and phase of each
    component field (E then B)."""
    rng = np.random.default_rng(seed)
    modes = []
    for _ in range(2):
        a = [np.array(_isotropic(rng, 1))[:, 0] * 10.0 ** rng.uniform(-3.5, -2.5) for _ in range(m)]
        k = [np.array(_isotropic(rng, 1))[:, 0] * 10.0 ** rng.uniform(-4.5, -3.5) for _ in range(m)]
        ph = rng.uniform(0.0, 2.0 * math.pi, m)
        modes.append((a, k, ph))
    return modes


def general_field_at(x, y, z, seed=21):
    """E(r) = sum_m a_m cos(k_m . r + phi_m), B likewise with its own modes: smooth,
    non-zero, E and B at general angles.  Positions as float64 arrays; returns the
    six per-slot field arrays."""
    out = {}
    for (a, k, ph), names in zip(_field_modes(seed), (("ex", "ey", "ez"), ("bx", "by", "bz"))):
        acc = np.zeros((3, np.size(x)))
        for am, km, pm in zip(a, k, ph):
            acc += am[:, None] * np.cos(km[0] * x + km[1] * y + km[2] * z + pm)[None, :]
        for j, nm in enumerate(names):
            out[nm] = np.ascontiguousarray(acc[j])
    return out


def general(n_e=24576, n_p=8192, n_g=8192, seed=22, field_seed=21):
    """Electrons, positrons and photons (gamma or photon energy log-uniform in
    [1e1, 10^3.5], isotropic) in the field of general_field_at at their positions."""
    rng = np.random.default_rng(seed)
    out = {}
    id0 = 0
    for name, n in (("electrons", n_e), ("positrons", n_p), ("photons", n_g)):
        s = _species(n, id0, rng)
        id0 += n
        energy = 10.0 ** rng.uniform(1.0, 3.5, n)
        u = energy if name == "photons" else np.sqrt(energy * energy - 1.0)
        dx, dy, dz = _isotropic(rng, n)
        s["ux"], s["uy"], s["uz"] = u * dx, u * dy, u * dz
        out[name] = s
    out.update({"field_seed": field_seed, "dt": DT_GENERAL, "seed": 1, "p_max": P_MAX})
    return out


def crossed(n=16384, seed=23, e0=1.0e-3):
    """Electrons in crossed fields just below the light-like limit: per particle a random
    orthonormal frame (e1, e2, e3), E = e0 e1, B = e0 (1 + eps) e2 with eps log-uniform
    in [1e-4, 1e-2], and u of magnitude log-uniform in [1e3, 10^4.5] along E x B = e3
    tilted by an angle log-uniform in [1e-5, 1e-3].  Returns the population and its
    per-slot fields."""
    rng = np.random.default_rng(seed)
    e = _species(n, 0, rng)
    e1 = np.stack(_isotropic(rng, n))
    r = np.stack(_isotropic(rng, n))
    e2 = np.cross(e1.T, r.T).T
    e2 /= np.linalg.norm(e2, axis=0)
    e3 = np.cross(e1.T, e2.T).T
    eps = 10.0 ** rng.uniform(-4.0, -2.0, n)
    tilt = 10.0 ** rng.uniform(-5.0, -3.0, n)
    az = rng.uniform(0.0, 2.0 * math.pi, n)
    umag = 10.0 ** rng.uniform(3.0, 4.5, n)
    d = e3 * np.cos(tilt) + (e1 * np.cos(az) + e2 * np.sin(az)) * np.sin(tilt)
    e["ux"], e["uy"], e["uz"] = umag * d[0], umag * d[1], umag * d[2]
    E = e0 * e1
    B = e0 * (1.0 + eps) * e2
    fields = {k: np.ascontiguousarray(v) for k, v in
              zip(("ex", "ey", "ez", "bx", "by", "bz"), (E[0], E[1], E[2], B[0], B[1], B[2]))}
    return {"electrons": e, "positrons": _empty(), "photons": _empty(), "fields": fields,
            "dt": DT_CROSSED, "seed": 1, "p_max": P_MAX}
