"""Grid coupling of the generator in FP64 (test infrastructure only): the PIC stages
around the push (Sec. 2.1, stage 2, field interpolation to the particles, and stage 4,
current deposition), on a periodic Cartesian Yee grid.

Grid: nx * ny * nz cells of size dx, dy, dz from the origin (x0, y0, z0); component
arrays are indexed [k, j, i] (i fastest in memory).  Each component sits at its Yee
position (fractions of a cell from node (i, j, k)):

    Ex, Jx (1/2, 0, 0)   Ey, Jy (0, 1/2, 0)   Ez, Jz (0, 0, 1/2)
    Bx (0, 1/2, 1/2)     By (1/2, 0, 1/2)     Bz (1/2, 1/2, 0)

Interpolation: linear (cloud-in-cell) in each direction on the component's own
lattice, periodic.  Deposition: every particle adds q w u / gamma (its current, with
u/gamma its velocity in units of c) times the same weights, divided by the cell
volume, to Jx, Jy, Jz.  Written as the definition, one particle and one corner at a
time (numpy over particles).  Cells (for sub-steps chosen per cell): the node cells
[x0 + i dx, x0 + (i + 1) dx) x ..., periodic.  Pinned in tests/test_oracle_grid.py and
tests/test_oracle_cells.py.
"""
from __future__ import annotations

import math

import numpy as np

STAGGER = {"ex": (0.5, 0.0, 0.0), "ey": (0.0, 0.5, 0.0), "ez": (0.0, 0.0, 0.5),
           "bx": (0.0, 0.5, 0.5), "by": (0.5, 0.0, 0.5), "bz": (0.5, 0.5, 0.0)}
J_STAGGER = {"jx": STAGGER["ex"], "jy": STAGGER["ey"], "jz": STAGGER["ez"]}


def _corners(grid, x, y, z, off):
    """For each particle: the 8 (flat index, weight) pairs of the lattice shifted by off."""
    n = np.array([grid["nx"], grid["ny"], grid["nz"]])
    s = [(np.asarray(p, np.float64) - grid[o]) / grid[d] - f
         for p, o, d, f in zip((x, y, z), ("x0", "y0", "z0"), ("dx", "dy", "dz"), off)]
    lo = [np.floor(c) for c in s]
    fr = [c - l for c, l in zip(s, lo)]
    out = []
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                i = (lo[0].astype(np.int64) + cx) % n[0]
                j = (lo[1].astype(np.int64) + cy) % n[1]
                k = (lo[2].astype(np.int64) + cz) % n[2]
                w = ((fr[0] if cx else 1.0 - fr[0]) * (fr[1] if cy else 1.0 - fr[1]) *
                     (fr[2] if cz else 1.0 - fr[2]))
                out.append(((k * n[1] + j) * n[0] + i, w))
    return out


def cell_index(grid, x, y, z):
    """Flat index (k ny + j) nx + i of the grid cell [x0 + i dx, x0 + (i + 1) dx) x (same in
    y, z) that holds each position, periodic (i = floor((x - x0) / dx) mod nx, exact integer
    arithmetic); -1 where a coordinate or (x - x0) / dx is not finite."""
    x, y, z = (np.atleast_1d(np.asarray(v, np.float64)) for v in (x, y, z))
    out = np.full(x.size, -1, np.int64)
    for p in range(x.size):
        idx = []
        for v, o, d, n in ((x[p], "x0", "dx", "nx"), (y[p], "y0", "dy", "ny"), (z[p], "z0", "dz", "nz")):
            s = (float(v) - grid[o]) / grid[d]
            if not math.isfinite(s):
                break
            idx.append(math.floor(s) % grid[n])
        if len(idx) == 3:
            out[p] = (idx[2] * grid["ny"] + idx[1]) * grid["nx"] + idx[0]
    return out


def gather(grid, x, y, z):
    """Stage 2: {component: values at the particles} for ex .. bz."""
    res = {}
    for c, off in STAGGER.items():
        f = np.asarray(grid[c], np.float64).ravel()
        res[c] = sum(w * f[idx] for idx, w in _corners(grid, x, y, z, off))
    return res


def deposit(grid, x, y, z, ux, uy, uz, w, charge):
    """Stage 4: (jx, jy, jz) flat arrays of the current density of the particles."""
    ncell = grid["nx"] * grid["ny"] * grid["nz"]
    vol = grid["dx"] * grid["dy"] * grid["dz"]
    u = [np.asarray(v, np.float64) for v in (ux, uy, uz)]
    gamma = np.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    out = {}
    for (c, off), uc in zip(J_STAGGER.items(), u):
        jc = np.zeros(ncell)
        q = charge * np.asarray(w, np.float64) * uc / gamma / vol
        for idx, wt in _corners(grid, x, y, z, off):
            np.add.at(jc, idx, q * wt)
        out[c] = jc
    return out["jx"], out["jy"], out["jz"]
