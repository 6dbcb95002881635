"""Pins of the oracle's in-step cascades: follow-up passes over the particles
created in the step, each running over the rest of the step from its birth time."""
import math

import numpy as np

import oracle


def _species(u, n, id0, dirn=(1.0, 0.0, 0.0)):
    d = np.asarray(dirn, np.float64) / np.linalg.norm(dirn)
    return {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n), "ux": np.full(n, u * d[0]),
            "uy": np.full(n, u * d[1]), "uz": np.full(n, u * d[2]), "w": np.ones(n),
            "id": np.arange(id0, id0 + n, dtype=np.uint64)}


def _empty():
    s = {k: np.zeros(0) for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
    s["id"] = np.zeros(0, np.uint64)
    return s


def _field(**kw):
    return {k: np.array([kw.get(k, 0.0)]) for k in ("ex", "ey", "ez", "bx", "by", "bz")}


def test_zero_generations_is_the_plain_step():
    f = _field(bz=1e-3)
    e = _species(5000.0, 300, 0)
    g = _species(3000.0, 100, 10_000, (0, 1, 0))
    dt = 3e4
    ee, pp, gg, _ = oracle.cascade_step(e, _empty(), g, f, dt, 3, 0, generations=0)
    e2 = {k: v.copy() for k, v in e.items()}
    g2 = {k: v.copy() for k, v in g.items()}
    chg, alive, _, _, _ = oracle.photon_step(g2, f, dt, 3, 0)
    che, _, _, _ = oracle.lepton_step(e2, f, -1.0, dt, 3, 0)
    assert np.array_equal(ee["ux"][:300], e2["ux"]) and np.array_equal(ee["x"][:300], e2["x"])
    assert np.array_equal(np.sort(gg["id"]), np.sort(np.concatenate([g2["id"][alive.astype(bool)], che["id"]])))
    assert ee["id"].size == 300 + int(np.sum(chg["kind"] == 1))


def test_children_run_the_rest_of_the_step():
    """Photons emitted in a weak B field cannot decay: in the follow-up pass each one
    moves by dir (dt - t_birth), its birth time being the end of the parent's sub-step."""
    f = _field(bz=1e-4)
    e = _species(2000.0, 400, 0)
    dt = 4e5
    ee, pp, gg, tallies = oracle.cascade_step(e, _empty(), _empty(), f, dt, 5, 2, generations=1)
    # the photons of the first pass, before and after the follow-up pass
    e0 = {k: v.copy() for k, v in e.items()}
    che, nsub, _, _ = oracle.lepton_step(e0, f, -1.0, dt, 5, 2)
    assert che["id"].size > 50
    assert np.all(che["tb"] > 0) and np.all(che["tb"] <= dt * (1 + 1e-12))
    # birth time = (sub-step index + 1) * dt / N of the parent
    par = {int(i): j for j, i in enumerate(e["id"])}
    st = dt / nsub[[par[int(p)] for p in che["parent"]]]
    assert np.allclose(che["tb"], (che["sub"] + 1.0) * st, rtol=1e-14, atol=0)
    pos = {int(i): j for j, i in enumerate(gg["id"])}
    k = np.stack([che["px"], che["py"], che["pz"]])
    d = k / np.linalg.norm(k, axis=0)
    for j in range(che["id"].size):
        jj = pos[int(che["id"][j])]
        moved = np.array([gg["x"][jj] - che["x"][j], gg["y"][jj] - che["y"][j], gg["z"][jj] - che["z"][j]])
        expect = d[:, j] * (dt - che["tb"][j])
        assert np.allclose(moved, expect, rtol=1e-10, atol=1e-9 * dt)
        assert gg["birth"][jj] == che["tb"][j]
    assert np.all(ee["birth"] == 0.0)
    # the follow-up pass ran exactly these photons
    assert tallies[1][0]["substeps"] >= che["id"].size


def test_cascade_creates_second_generation_pairs():
    """Strong field, very energetic electrons: photons emitted early in the step decay
    into pairs within the same step; every child is born after its parent started."""
    f = _field(bz=2e-3)
    e = _species(2e5, 1000, 0)
    dt = 1e5
    ee, pp, gg, tallies = oracle.cascade_step(e, _empty(), _empty(), f, dt, 9, 0, generations=2)
    assert pp["id"].size > 0                       # pairs created inside the step
    assert tallies[1][0]["events"] == pp["id"].size
    assert ee["id"].size == 1000 + pp["id"].size
    # without cascades the same step has no pairs
    _, pp0, _, _ = oracle.cascade_step(e, _empty(), _empty(), f, dt, 9, 0, generations=0)
    assert pp0["id"].size == 0


def test_event_gap_histogram_definition():
    """Gaps: the first event of a particle counts the sub-steps since the step start, the
    next ones the sub-steps since its previous event; pairs count from the step start."""
    ch = {"parent": np.array([7, 7, 3, 7, 3], np.uint64), "sub": np.array([4, 0, 2, 9, 30], np.uint32)}
    ph = {"kind": np.array([1, 2, 1, 2], np.int32), "sub": np.array([0, 0, 5, 5], np.uint32)}
    he, hp = oracle.event_gaps([ch], ph, 16)
    # particle 7: subs 0, 4, 9 -> gaps 1, 4, 5; particle 3: subs 2, 30 -> gaps 3, 28 (last bin)
    exp = np.zeros(16, np.int64)
    for gp in (1, 4, 5, 3, 15):
        exp[gp] += 1
    assert np.array_equal(he, exp)
    assert hp[1] == 1 and hp[6] == 1 and hp.sum() == 2


def test_event_gaps_of_an_oracle_step_sum_to_its_events():
    f = _field(bz=1e-3)
    e = _species(3000.0, 500, 0)
    ch, nsub, nev, tl = oracle.lepton_step(e, f, -1.0, 3e5, 2, 0)
    he, _ = oracle.event_gaps([ch], None, 32)
    assert he.sum() == nev.sum() == ch["id"].size
    # with N sub-steps no gap exceeds N
    assert he[int(nsub.max()) + 1:].sum() == 0 or nsub.max() + 1 >= 32
