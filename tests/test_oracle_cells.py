"""Pins of the oracle's sub-steps chosen per cell (Algorithms 1 and 2, step 1, read for
the current cell): own_substeps is the count the oracle's own step takes, cell_index
puts a position into the cell it was built in, a cell's count is the largest of its
lepton (or photon) group, and a particle run with its cell's finer sub-step emits at
the same rate."""
import math

import numpy as np

import oracle
import workloads
from oracle import grid as og

CELLS = {"nx": 5, "ny": 3, "nz": 4, "dx": 2.0e3, "dy": 1.5e3, "dz": 2.5e3, "x0": -1.0e3, "y0": 4.0e2, "z0": -6.0e3}


def _at_cells(sp, ijk, frac):
    """Place particle p at x0 + (i + f) dx etc., i possibly outside the box."""
    for p, ((i, j, k), f) in enumerate(zip(ijk, frac)):
        sp["x"][p] = CELLS["x0"] + (i + f[0]) * CELLS["dx"]
        sp["y"][p] = CELLS["y0"] + (j + f[1]) * CELLS["dy"]
        sp["z"][p] = CELLS["z0"] + (k + f[2]) * CELLS["dz"]


def test_own_substeps_equal_the_steps_own_count():
    w = workloads.c1(n=400, seed=3)
    st = {k: v.copy() for k, v in w["electrons"].items()}
    own = oracle.own_substeps(st, w["fields"], w["dt"])
    _, nsub, _, _ = oracle.lepton_step(st, w["fields"], -1.0, w["dt"], 1, 0, threads=1)
    assert np.array_equal(own, nsub) and own.min() >= 1
    c2 = workloads.c2(n_e=300, n_g=300, seed=4)
    fg = workloads.c2_field(0)
    ph = {k: v.copy() for k, v in c2["photons"].items()}
    own = oracle.own_substeps(ph, fg, c2["dt"], photons=True)
    _, _, nsub, nev, _ = oracle.photon_step(ph, fg, c2["dt"], 1, 0, threads=1)
    # a photon that decays stops early; the others run their whole count
    assert np.array_equal(own[nev == 0], nsub[nev == 0]) and np.all(nsub[nev == 1] <= own[nev == 1])


def test_cell_index_by_construction():
    rng = np.random.default_rng(1)
    n = 500
    ijk = rng.integers(-7, 12, size=(n, 3))
    frac = rng.uniform(0.01, 0.99, size=(n, 3))
    sp = {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n)}
    _at_cells(sp, ijk, frac)
    got = og.cell_index(CELLS, sp["x"], sp["y"], sp["z"])
    i, j, k = ijk[:, 0] % CELLS["nx"], ijk[:, 1] % CELLS["ny"], ijk[:, 2] % CELLS["nz"]
    assert np.array_equal(got, (k * CELLS["ny"] + j) * CELLS["nx"] + i)
    assert og.cell_index(CELLS, [np.nan, 0.0, np.inf], [0.0, 0.0, 0.0], [0.0, np.nan, 0.0]).tolist() == [-1, -1, -1]


def _population(n, seed):
    w = workloads.c1(n=n, seed=seed)
    return {k: v.copy() for k, v in w["electrons"].items()}, w


def test_one_particle_per_cell_is_the_per_particle_step():
    n = CELLS["nx"] * CELLS["ny"] * CELLS["nz"]
    e, w = _population(n, 5)
    ijk = [(i, j, k) for k in range(CELLS["nz"]) for j in range(CELLS["ny"]) for i in range(CELLS["nx"])]
    _at_cells(e, ijk, np.full((n, 3), 0.5))
    empty = {k: np.zeros(0) for k in e}
    empty["id"] = np.zeros(0, np.uint64)
    forced = oracle.cell_substeps(e, empty, empty, [w["fields"]] * 3, CELLS, w["dt"])
    own = oracle.own_substeps(e, w["fields"], w["dt"])
    assert np.array_equal(forced[0], own)
    a, b = {k: v.copy() for k, v in e.items()}, {k: v.copy() for k, v in e.items()}
    ca, na, ea, _ = oracle.lepton_step(a, w["fields"], -1.0, w["dt"], 2, 0, threads=1)
    cb, nb, eb, _ = oracle.lepton_step(b, w["fields"], -1.0, w["dt"], 2, 0, threads=1, nsub=forced[0])
    assert np.array_equal(na, nb) and np.array_equal(ea, eb)
    assert np.array_equal(ca["id"], cb["id"]) and all(np.array_equal(a[k], b[k]) for k in a)


def test_cell_count_is_the_largest_of_its_group():
    """Cell A holds an electron of large chi and a positron of small chi: both take the
    electron's count; the photon in A keeps its own (its group is separate); the
    electron alone in cell B keeps its own."""
    def sp(n):
        return {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n), "ux": np.zeros(n), "uy": np.zeros(n),
                "uz": np.zeros(n), "w": np.ones(n), "id": np.arange(n, dtype=np.uint64)}
    e, p, g = sp(2), sp(1), sp(1)
    f = workloads.uniform_field(bz=2e-3)
    e["ux"][0], e["uz"][1] = 1e3, 1e4   # chi 2, and moving along B (chi 0)
    p["uz"][:] = [1e4]
    g["uz"][:] = [5e3]
    _at_cells(e, [(1, 1, 1), (3, 0, 2)], [(0.2, 0.3, 0.4), (0.5, 0.5, 0.5)])
    _at_cells(p, [(1 + CELLS["nx"], 1, 1)], [(0.9, 0.1, 0.6)])       # cell A, one period away
    _at_cells(g, [(1, 1, 1)], [(0.5, 0.5, 0.5)])
    own = [oracle.own_substeps(s, f, 1e4, photons=(k == 2)) for k, s in enumerate((e, p, g))]
    ne, np_, ng = oracle.cell_substeps(e, p, g, [f] * 3, CELLS, 1e4)
    assert own[0][0] > 4 * max(own[0][1], own[1][0], own[2][0])
    assert ne.tolist() == [own[0][0], own[0][1]]
    assert np_.tolist() == [own[0][0]]
    assert ng.tolist() == [own[2][0]]
    # a non-finite position keeps the particle's own count and joins no cell
    e["x"][0] = np.nan
    ne, np_, _ = oracle.cell_substeps(e, p, g, [f] * 3, CELLS, 1e4)
    assert ne[0] == own[0][0] and np_[0] == own[1][0]


def test_finer_cell_substeps_keep_the_emission_rate():
    """Electrons in one cell, one of them in a field 500 times stronger: everyone runs
    its cell's count (over 100 times its own), the emission count stays that of the
    per-particle step (4.5 sigma), and the step takes exactly the forced counts."""
    n = 30000
    rng = np.random.default_rng(7)
    gamma = 10.0 ** rng.uniform(3.0, 3.5, n)
    gamma[0] = 100.0
    e = {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n), "ux": np.sqrt(gamma ** 2 - 1), "uy": np.zeros(n),
         "uz": np.zeros(n), "w": np.ones(n), "id": np.arange(n, dtype=np.uint64)}
    f = {k: np.zeros(n) for k in ("ex", "ey", "ez", "bx", "by", "bz")}
    f["bz"][:] = 1e-2
    f["bz"][0] = 5.0
    dt = 600.0
    empty = {k: np.zeros(0) for k in e}
    empty["id"] = np.zeros(0, np.uint64)
    forced = oracle.cell_substeps(e, empty, empty, [f, f, f], {**CELLS, "nx": 1, "ny": 1, "nz": 1}, dt)[0]
    own = oracle.own_substeps(e, f, dt)
    assert np.all(forced == own[0]) and forced[1:].mean() > 100 * own[1:].mean()
    a, b = {k: v.copy() for k, v in e.items()}, {k: v.copy() for k, v in e.items()}
    _, _, ea, ta = oracle.lepton_step(a, f, -1.0, dt, 3, 0)
    _, nb, eb, tb = oracle.lepton_step(b, f, -1.0, dt, 3, 0, nsub=forced)
    assert np.array_equal(nb, forced) and tb["substeps"] == int(forced.sum())
    na, nbv = int(ea[1:].sum()), int(eb[1:].sum())
    assert na > 500
    assert abs(na - nbv) <= 4.5 * math.sqrt(na + nbv), (na, nbv)
