"""Pins of the oracle's grid coupling (field interpolation and current deposition on a
periodic Yee grid): linear fields are interpolated exactly, interpolation is periodic,
a particle on a component's node picks that node's value, and the deposited current
integrates to the particles' total current."""
import numpy as np

from oracle import grid as og


def _grid(nx=5, ny=4, nz=6, d=(0.7, 1.1, 0.9), origin=(-1.0, 0.5, 2.0)):
    return {"nx": nx, "ny": ny, "nz": nz, "dx": d[0], "dy": d[1], "dz": d[2],
            "x0": origin[0], "y0": origin[1], "z0": origin[2]}


def _positions(g, component):
    """Physical positions of every node of a component's lattice, [k, j, i] order."""
    off = og.STAGGER.get(component) or og.J_STAGGER[component]
    k, j, i = np.meshgrid(np.arange(g["nz"]), np.arange(g["ny"]), np.arange(g["nx"]), indexing="ij")
    return (g["x0"] + (i + off[0]) * g["dx"], g["y0"] + (j + off[1]) * g["dy"], g["z0"] + (k + off[2]) * g["dz"])


def test_linear_fields_interpolate_exactly():
    """Each component a x + b y + c z + e on its own lattice: inside the box (no wrap) linear
    interpolation returns the same linear function at any point."""
    g = _grid()
    coef = {c: np.random.default_rng(i).normal(size=4) for i, c in enumerate(og.STAGGER)}
    for c in og.STAGGER:
        X, Y, Z = _positions(g, c)
        a = coef[c]
        g[c] = a[0] * X + a[1] * Y + a[2] * Z + a[3]
    rng = np.random.default_rng(5)
    # points at least one cell from the far faces, so no corner wraps
    x = g["x0"] + rng.uniform(0.5, g["nx"] - 1.5, 200) * g["dx"]
    y = g["y0"] + rng.uniform(0.5, g["ny"] - 1.5, 200) * g["dy"]
    z = g["z0"] + rng.uniform(0.5, g["nz"] - 1.5, 200) * g["dz"]
    got = og.gather(g, x, y, z)
    for c in og.STAGGER:
        a = coef[c]
        assert np.allclose(got[c], a[0] * x + a[1] * y + a[2] * z + a[3], rtol=1e-12, atol=1e-12)


def test_nodes_and_periodicity():
    g = _grid()
    rng = np.random.default_rng(2)
    for c in og.STAGGER:
        g[c] = rng.normal(size=(g["nz"], g["ny"], g["nx"]))
    for c in og.STAGGER:
        X, Y, Z = _positions(g, c)
        assert np.allclose(og.gather(g, X.ravel(), Y.ravel(), Z.ravel())[c], g[c].ravel(), rtol=0, atol=1e-12)
    # shifting by whole periods changes nothing
    x, y, z = rng.uniform(-3, 3, 50), rng.uniform(-3, 3, 50), rng.uniform(-3, 3, 50)
    a = og.gather(g, x, y, z)
    b = og.gather(g, x + 2 * g["nx"] * g["dx"], y - g["ny"] * g["dy"], z + 3 * g["nz"] * g["dz"])
    for c in og.STAGGER:
        assert np.allclose(a[c], b[c], rtol=1e-12, atol=1e-12)
    # a uniform field is reproduced everywhere
    for c in og.STAGGER:
        g[c] = np.full((g["nz"], g["ny"], g["nx"]), 0.37)
    assert all(np.allclose(v, 0.37) for v in og.gather(g, x, y, z).values())


def test_deposit_conserves_total_current():
    """sum(J) dV = sum q w u / gamma, per component, for any positions (the weights of a
    particle sum to one); a particle on a Jx node puts all its x-current there."""
    g = _grid()
    rng = np.random.default_rng(3)
    n = 300
    x, y, z = rng.uniform(-5, 5, n), rng.uniform(-5, 5, n), rng.uniform(-5, 5, n)
    ux, uy, uz = rng.normal(size=n) * 10, rng.normal(size=n) * 10, rng.normal(size=n) * 10
    w = rng.uniform(0.5, 2.0, n)
    jx, jy, jz = og.deposit(g, x, y, z, ux, uy, uz, w, -1.0)
    gam = np.sqrt(1 + ux ** 2 + uy ** 2 + uz ** 2)
    vol = g["dx"] * g["dy"] * g["dz"]
    for j, u in ((jx, ux), (jy, uy), (jz, uz)):
        assert np.isclose(j.sum() * vol, np.sum(-w * u / gam), rtol=1e-12)
    X, Y, Z = _positions(g, "jx")
    jx1, _, _ = og.deposit(g, [X[2, 1, 3]], [Y[2, 1, 3]], [Z[2, 1, 3]], [3.0], [0.0], [0.0], [1.0], 1.0)
    k = (2 * g["ny"] + 1) * g["nx"] + 3
    assert np.isclose(jx1[k], 3.0 / np.sqrt(10.0) / vol)
    assert np.abs(np.delete(jx1, k)).max() < 1e-12 * jx1[k]   # rounding of the node position only
