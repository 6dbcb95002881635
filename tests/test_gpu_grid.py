"""Grid coupling on the GPU (qed_gather, qed_deposit) against the oracle's definition:
interpolation of every Yee component to the particles, deposition of their currents,
both periodic; and one PIC cycle (gather, step, deposit) with the total current of the
grid equal to the particles'."""
import numpy as np
import pytest

import workloads
from oracle import grid as og

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

COMP = ("ex", "ey", "ez", "bx", "by", "bz")


def _grid(qed, real, rng, nx=17, ny=9, nz=12, scale=1e-3):
    g = {"nx": nx, "ny": ny, "nz": nz, "dx": 0.8, "dy": 1.3, "dz": 1.1, "x0": -3.0, "y0": 2.0, "z0": -7.5}
    dev = {}
    for c in COMP:
        v = rng.normal(size=(nz, ny, nx)) * scale
        t = torch.from_numpy(v).to(real).cuda()
        dev[c] = t
        g[c] = t.double().cpu().numpy()          # the values as the GPU holds them
    s = qed.qed_grid()
    for c in COMP:
        setattr(s, c, dev[c].data_ptr())
    s.nx, s.ny, s.nz = nx, ny, nz
    for k in ("x0", "y0", "z0", "dx", "dy", "dz"):
        setattr(s, k, g[k])
    return g, s, dev


def _particles(g, rng, n):
    # positions inside and outside the box (periodic), momenta of all directions
    span = np.array([g["nx"] * g["dx"], g["ny"] * g["dy"], g["nz"] * g["dz"]])
    x = g["x0"] + rng.uniform(-1.0, 2.0, n) * span[0]
    y = g["y0"] + rng.uniform(-1.0, 2.0, n) * span[1]
    z = g["z0"] + rng.uniform(-1.0, 2.0, n) * span[2]
    u = rng.normal(size=(3, n)) * 30.0
    return {"x": x, "y": y, "z": z, "ux": u[0], "uy": u[1], "uz": u[2], "w": rng.uniform(0.5, 2.0, n),
            "id": np.arange(n, dtype=np.uint64)}


@pytest.mark.parametrize("prec_name", ["F64", "MIXED"])
def test_gather_matches_oracle(prec_name):
    from paper_2008_10468_amd import qed
    prec = getattr(qed, "QED_PREC_" + prec_name)
    rng = np.random.default_rng(1)
    gen = qed.Generator(precision=prec, capacity=(50000, 16, 16))
    g, s, dev = _grid(qed, gen.real, rng)
    p = _particles(g, rng, 40000)
    gen.sp[0].upload(p)
    out = [torch.full((50000,), float("nan"), dtype=gen.real, device="cuda") for _ in COMP]
    assert qed.qed_gather(gen.ctx, s, gen.sp[0].struct(), [t.data_ptr() for t in out]) == qed.QED_OK
    torch.cuda.synchronize()
    ref = og.gather(g, p["x"], p["y"], p["z"])
    tol = 1e-12 if prec_name == "F64" else 2e-6
    for c, t in zip(COMP, out):
        got = t.double().cpu().numpy()
        assert np.all(np.isnan(got[40000:]))                     # slots past the count untouched
        err = np.abs(got[:40000] - ref[c]).max() / np.abs(g[c]).max()
        assert err < tol, (c, err)
    gen.close()


SORT = {"sorted": 0, "wave": 0xFFFFFFFF}   # qed_tuning.deposit_sort_min: always / never


def _deposit_mode(qed, gen, mode):
    t = qed.qed_get_tuning(gen.ctx)
    t.deposit_sort_min = SORT[mode]
    assert qed.qed_set_tuning(gen.ctx, t) == qed.QED_OK


def _deposit_check(qed, gen, g, s, charge=-1.0):
    """qed_deposit of species 0 against the oracle on the stored values (1e-10 of the
    largest current)."""
    q = gen.sp[0].download()                                     # momenta and weights as stored
    ncell = g["nx"] * g["ny"] * g["nz"]
    j = [torch.zeros(ncell, dtype=torch.float64, device="cuda") for _ in range(3)]
    assert qed.qed_deposit(gen.ctx, s, gen.sp[0].struct(), charge, *[t.data_ptr() for t in j]) == qed.QED_OK
    torch.cuda.synchronize()
    ref = og.deposit(g, q["x"], q["y"], q["z"], q["ux"], q["uy"], q["uz"], q["w"], charge)
    for t, r in zip(j, ref):
        got = t.cpu().numpy()
        assert np.abs(got - r).max() <= 1e-10 * max(np.abs(r).max(), 1e-300)
    return j


def test_gather_benchmark_size():
    """The grid benchmark's gather: the 1,048,576 C2 electrons in random order, a 32^3 grid
    of float fields, against the oracle on a sample of 2^16 particles (2e-6 of the largest
    field value)."""
    from paper_2008_10468_amd import qed
    n = 1 << 20
    w = workloads.c2(n_e=n, n_g=16)
    geom = workloads.cell_box(32)
    gen = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, 16, 16), parent=False, events=False)
    gen.sp[0].upload(w["electrons"])
    rng = np.random.default_rng(5)
    g = dict(geom)
    dev = {}
    for c in COMP:
        v = rng.normal(size=(32, 32, 32)) * 1e-3
        dev[c] = torch.from_numpy(v).float().cuda()
        g[c] = dev[c].double().cpu().numpy()
    s = qed.cell_geometry(geom)
    for c in COMP:
        setattr(s, c, dev[c].data_ptr())
    out = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in COMP]
    assert qed.qed_gather(gen.ctx, s, gen.sp[0].struct(), [t.data_ptr() for t in out]) == qed.QED_OK
    torch.cuda.synchronize()
    e = gen.sp[0].download()
    idx = np.sort(rng.choice(n, 1 << 16, replace=False))
    ref = og.gather(g, e["x"][idx], e["y"][idx], e["z"][idx])
    for c, t in zip(COMP, out):
        got = t.double().cpu().numpy()[idx]
        assert np.abs(got - ref[c]).max() <= 2e-6 * np.abs(g[c]).max(), c
    gen.close()


@pytest.mark.parametrize("mode", ["sorted", "wave"])
@pytest.mark.parametrize("prec_name", ["F64", "MIXED"])
def test_deposit_matches_oracle(prec_name, mode):
    from paper_2008_10468_amd import qed
    prec = getattr(qed, "QED_PREC_" + prec_name)
    rng = np.random.default_rng(2)
    gen = qed.Generator(precision=prec, capacity=(70000, 16, 16))   # slots past the count ignored
    _deposit_mode(qed, gen, mode)
    g, s, _ = _grid(qed, gen.real, rng, nx=11, ny=7, nz=5)
    gen.sp[0].upload(_particles(g, rng, 60000))
    _deposit_check(qed, gen, g, s)
    gen.close()


def _clustered(g, rng, n, frac, lo, hi):
    """Particles uniform over the box, a fraction of them inside the cell box [lo, hi)."""
    p = _particles(g, rng, n)
    k = int(n * frac)
    d = {"x": "dx", "y": "dy", "z": "dz"}
    for a, (l, h) in zip("xyz", zip(lo, hi)):
        p[a][:k] = g[a + "0"] + rng.uniform(l, h, k) * g[d[a]]
    perm = rng.permutation(n)
    return {key: v[perm] for key, v in p.items()}


@pytest.mark.parametrize("case", ["sparse", "many_tiles", "clustered", "tiny_grid", "cell_order", "one", "empty"])
def test_deposit_sorted_cases(case):
    """The tile-sorted deposition on each of its branches: tiles summed in LDS (dense),
    particles added directly (tiles of fewer than 256), both within one chunk
    (clustered), tiles counted with global atomics (more than 4096 tiles), grids of
    fewer cells than a tile along an axis, particles in cell order (all lanes of a wave
    on the same LDS points), a single particle and none."""
    from paper_2008_10468_amd import qed
    rng = np.random.default_rng(31)
    shape, n = {"sparse": ((64, 32, 16), 20000), "many_tiles": ((84, 80, 52), 100000),
                "clustered": ((32, 24, 20), 60000), "tiny_grid": ((1, 2, 3), 30000),
                "cell_order": ((16, 12, 8), 50000), "one": ((9, 9, 9), 1), "empty": ((9, 9, 9), 0)}[case]
    gen = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(max(n, 64) + 100, 16, 16))
    _deposit_mode(qed, gen, "sorted")
    g, s, _ = _grid(qed, gen.real, rng, nx=shape[0], ny=shape[1], nz=shape[2])
    if case == "clustered":
        p = _clustered(g, rng, n, 0.5, (4.0, 8.0, 0.0), (12.0, 12.0, 4.0))   # two tiles
    else:
        p = _particles(g, rng, n)
    if case == "cell_order":
        cell = ((np.floor((p["z"] - g["z0"]) / g["dz"]) % g["nz"]) * g["ny"] +
                (np.floor((p["y"] - g["y0"]) / g["dy"]) % g["ny"])) * g["nx"] + \
            (np.floor((p["x"] - g["x0"]) / g["dx"]) % g["nx"])
        order = np.argsort(cell, kind="stable")
        p = {k: v[order] for k, v in p.items()}
    gen.sp[0].upload(p)
    j = _deposit_check(qed, gen, g, s, charge=1.0)
    if n == 0:
        assert all(float(t.abs().max()) == 0.0 for t in j)
    gen.close()


@pytest.mark.parametrize("order", ["random", "cell"])
def test_deposit_benchmark_size(order):
    """The grid benchmark's configuration: the 1,048,576 C2 electrons in a periodic box of
    32^3 cells (32 per cell), mixed precision, the default (tile-sorted) deposit, in the
    order the benchmark times: against the oracle to 1e-10 of the largest current."""
    from paper_2008_10468_amd import qed
    n = 1 << 20
    w = workloads.c2(n_e=n, n_g=16)
    geom = workloads.cell_box(32)
    e = w["electrons"]
    if order == "cell":
        cell = ((np.floor((e["z"] - geom["z0"]) / geom["dz"]).astype(np.int64) % 32) * 32 +
                (np.floor((e["y"] - geom["y0"]) / geom["dy"]).astype(np.int64) % 32)) * 32 + \
            (np.floor((e["x"] - geom["x0"]) / geom["dx"]).astype(np.int64) % 32)
        e = workloads.subset(e, np.argsort(cell, kind="stable"))
    gen = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, 16, 16), parent=False, events=False)
    gen.sp[0].upload(e)
    g = dict(geom)
    print("deposit at the benchmark's size,", order, "order", flush=True)
    _deposit_check(qed, gen, g, qed.cell_geometry(geom))
    gen.close()


def test_deposit_in_a_recorded_graph():
    """qed_deposit recorded into a HIP graph: on a fresh context (no scratch yet, and none
    may be allocated while recording) it records the per-wave kernel; once the sorted
    deposit's scratch exists it records the sorted kernels.  Both graphs, replayed three
    times with eager work and a cleared current between the replays, give the oracle's
    current each time."""
    from paper_2008_10468_amd import qed
    rng = np.random.default_rng(41)
    stream = torch.cuda.Stream()
    gen = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(70000, 16, 16), stream=stream.cuda_stream)
    _deposit_mode(qed, gen, "sorted")
    g, s, _ = _grid(qed, gen.real, rng, nx=13, ny=9, nz=7)
    gen.sp[0].upload(_particles(g, rng, 60000))
    torch.cuda.synchronize()
    q = gen.sp[0].download()
    ref = og.deposit(g, q["x"], q["y"], q["z"], q["ux"], q["uy"], q["uz"], q["w"], -1.0)
    ncell = g["nx"] * g["ny"] * g["nz"]
    j = [torch.zeros(ncell, dtype=torch.float64, device="cuda") for _ in range(3)]
    ptrs = [t.data_ptr() for t in j]
    for case in ("fresh", "with_scratch"):
        if case == "with_scratch":     # an eager call outside the graph allocates the scratch
            assert qed.qed_deposit(gen.ctx, s, gen.sp[0].struct(), -1.0, *ptrs) == qed.QED_OK
            assert gen.sync()[0] == qed.QED_OK
        assert qed.qed_graph_begin(gen.ctx) == qed.QED_OK
        assert qed.qed_deposit(gen.ctx, s, gen.sp[0].struct(), -1.0, *ptrs) == qed.QED_OK
        st, graph = qed.qed_graph_end(gen.ctx)
        assert st == qed.QED_OK
        for rep in range(3):
            for t in j:
                t.zero_()
            junk = torch.randn(1 << 18, device="cuda").sum().item()
            torch.cuda.synchronize()
            assert qed.qed_graph_launch(gen.ctx, graph) == qed.QED_OK
            assert gen.sync()[0] == qed.QED_OK
            torch.cuda.synchronize()
            for t, r in zip(j, ref):
                assert np.abs(t.cpu().numpy() - r).max() <= 1e-10 * np.abs(r).max(), (case, rep)
        qed.qed_graph_destroy(graph)
    gen.close()


def test_deposit_sorted_changing_grids():
    """One context, grids of 12, 5460 and again 12 tiles (the scratch grows; the tile
    counts start from zero on every call) and a species that shrinks between calls."""
    from paper_2008_10468_amd import qed
    rng = np.random.default_rng(32)
    gen = qed.Generator(precision=qed.QED_PREC_F64, capacity=(80000, 16, 16))
    _deposit_mode(qed, gen, "sorted")
    for (nx, ny, nz), n in (((11, 7, 5), 80000), ((84, 80, 52), 50000), ((11, 7, 5), 30000)):
        g, s, _ = _grid(qed, gen.real, rng, nx=nx, ny=ny, nz=nz)
        gen.sp[0].upload(_particles(g, rng, n))
        _deposit_check(qed, gen, g, s)
    gen.close()


def test_pic_cycle_gather_step_deposit():
    """One PIC cycle on the C2 population placed in a grid holding C2's field: gather,
    a generator step with the gathered per-slot fields, deposition of the electrons'
    currents; the grid's total current equals the particles' (weights sum to one)."""
    from paper_2008_10468_amd import qed
    w = workloads.c2(n_e=30000, n_g=8000, seed=9)
    gen = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 16, 1 << 15, 1 << 17))
    gen.load_state({k: w[k] for k in ("electrons", "positrons", "photons")})
    rng = np.random.default_rng(3)
    nx, ny, nz = 16, 16, 16
    gd = {"nx": nx, "ny": ny, "nz": nz, "dx": 2e3, "dy": 2e3, "dz": 2e3, "x0": -1.6e4, "y0": -1.6e4, "z0": -1.6e4}
    dev = {c: torch.full((nz, ny, nx), float(w["fields"][c][0]), dtype=torch.float32, device="cuda") for c in COMP}
    s = qed.qed_grid()
    for c in COMP:
        setattr(s, c, dev[c].data_ptr())
    s.nx, s.ny, s.nz = nx, ny, nz
    for k in ("x0", "y0", "z0", "dx", "dy", "dz"):
        setattr(s, k, gd[k])
    # per-slot fields of every species from the grid
    per = []
    for sp in gen.sp:
        arrs = [torch.empty(sp.capacity, dtype=torch.float32, device="cuda") for _ in COMP]
        assert qed.qed_gather(gen.ctx, s, sp.struct(), [t.data_ptr() for t in arrs]) == qed.QED_OK
        f = qed.qed_field()
        for c, t in zip(COMP, arrs):
            setattr(f, c, t.data_ptr())
        f.stride = 1
        per.append((f, arrs))
    torch.cuda.synchronize()
    # a uniform grid field interpolates to the uniform value
    e0 = per[0][1][0][:30000].double().cpu().numpy()
    assert np.allclose(e0, w["fields"]["ex"][0], rtol=1e-6)
    assert qed.qed_step(gen.ctx, gen.particles(), [per[0][0], per[1][0], per[2][0]], w["dt"], 1, 0) == qed.QED_OK
    assert gen.sync()[0] == qed.QED_OK
    ncell = nx * ny * nz
    j = [torch.zeros(ncell, dtype=torch.float64, device="cuda") for _ in range(3)]
    assert qed.qed_deposit(gen.ctx, s, gen.sp[0].struct(), -1.0, *[t.data_ptr() for t in j]) == qed.QED_OK
    torch.cuda.synchronize()
    e = gen.sp[0].download()
    gam = np.sqrt(1 + e["ux"] ** 2 + e["uy"] ** 2 + e["uz"] ** 2)
    vol = gd["dx"] * gd["dy"] * gd["dz"]
    for t, u in zip(j, ("ux", "uy", "uz")):
        total = t.cpu().numpy().sum() * vol
        assert np.isclose(total, np.sum(-e["w"] * e[u] / gam), rtol=1e-9)
    gen.close()


def test_grid_rejects_bad_arguments():
    from paper_2008_10468_amd import qed
    gen = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(16, 16, 16))
    rng = np.random.default_rng(4)
    g, s, dev = _grid(qed, gen.real, rng, nx=4, ny=4, nz=4)
    out = [torch.empty(16, dtype=torch.float32, device="cuda") for _ in COMP]
    ptrs = [t.data_ptr() for t in out]
    s.dx = 0.0
    assert qed.qed_gather(gen.ctx, s, gen.sp[0].struct(), ptrs) == qed.QED_ERR_INVALID_ARG
    s.dx = 1.0
    s.nz = 0
    assert qed.qed_gather(gen.ctx, s, gen.sp[0].struct(), ptrs) == qed.QED_ERR_INVALID_ARG
    s.nz = 4
    assert qed.qed_gather(gen.ctx, s, gen.sp[0].struct(), ptrs[:5] + [None]) == qed.QED_ERR_INVALID_ARG
    assert qed.qed_deposit(gen.ctx, s, gen.sp[0].struct(), float("nan"), ptrs[0], ptrs[1], ptrs[2]) == \
        qed.QED_ERR_INVALID_ARG
    gen.close()


@pytest.mark.parametrize("mode", ["sorted", "wave"])
def test_non_finite_positions(mode):
    """A particle whose position is not finite gets NaN fields and deposits nothing;
    the others are unaffected (against the oracle on the finite particles)."""
    from paper_2008_10468_amd import qed
    rng = np.random.default_rng(6)
    gen = qed.Generator(precision=qed.QED_PREC_F64, capacity=(4096, 16, 16))
    _deposit_mode(qed, gen, mode)
    g, s, _ = _grid(qed, gen.real, rng, nx=9, ny=6, nz=5)
    p = _particles(g, rng, 4000)
    bad = np.zeros(4000, bool)
    bad[[3, 100, 2500]] = True
    p["x"][3], p["y"][100], p["z"][2500] = np.nan, np.inf, -np.inf
    p["x"][7] = 1e300                                       # finite but far away: wraps
    gen.sp[0].upload(p)
    out = [torch.empty(4096, dtype=gen.real, device="cuda") for _ in COMP]
    assert qed.qed_gather(gen.ctx, s, gen.sp[0].struct(), [t.data_ptr() for t in out]) == qed.QED_OK
    ncell = g["nx"] * g["ny"] * g["nz"]
    j = [torch.zeros(ncell, dtype=torch.float64, device="cuda") for _ in range(3)]
    assert qed.qed_deposit(gen.ctx, s, gen.sp[0].struct(), 1.0, *[t.data_ptr() for t in j]) == qed.QED_OK
    torch.cuda.synchronize()
    ok = ~bad
    ok[7] = False                                           # beyond 2^53 cells only kept in range
    ref = og.gather(g, p["x"][ok], p["y"][ok], p["z"][ok])
    for c, t in zip(COMP, out):
        got = t.cpu().numpy()[:4000]
        assert np.all(np.isnan(got[bad])) and np.isfinite(got[7])
        assert np.abs(got[ok] - ref[c]).max() <= 1e-12 * np.abs(g[c]).max()
    keep = ~bad
    q = {k: v[keep] for k, v in p.items()}
    # the far particle deposits somewhere in the box: compare the totals
    gam = np.sqrt(1 + q["ux"] ** 2 + q["uy"] ** 2 + q["uz"] ** 2)
    vol = g["dx"] * g["dy"] * g["dz"]
    for t, u in zip(j, ("ux", "uy", "uz")):
        got = t.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.isclose(got.sum() * vol, np.sum(q["w"] * q[u] / gam), rtol=1e-9)
    gen.close()
