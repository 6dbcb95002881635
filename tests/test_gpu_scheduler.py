"""The binned scheduler (sub-step-count bins, persistent heavy queue) gives the same
per-particle results as the naive one-lane-per-particle kernel, for any launch
shape, and matches the oracle."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import as_precision

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _sorted(d):
    o = np.argsort(d["id"])
    return {k: v[o] for k, v in d.items()}


def _run(w, sched, tuning=None, steps=3, precision=None, fields_fn=None, per_species=None):
    from paper_2008_10468_amd import qed
    precision = qed.QED_PREC_MIXED if precision is None else precision
    g = qed.Generator(precision=precision, capacity=(1 << 16, 1 << 15, 1 << 17), scheduler=sched)
    if tuning:
        t = qed.qed_get_tuning(g.ctx)
        for k, v in tuning.items():
            setattr(t, k, v)
        assert qed.qed_set_tuning(g.ctx, t) == qed.QED_OK
    g.load_state(w)
    for s in range(steps):
        if per_species is not None:
            g.set_fields(None, per_species=per_species)
        else:
            g.set_fields(fields_fn(s))
        g.step(w["dt"], 5, s)
        st, rep = g.sync()
        assert st == qed.QED_OK
    out = [_sorted(g.sp[k].download()) for k in range(3)]
    stats = g.stats()
    g.close()
    return out, stats


@pytest.mark.parametrize("tuning", [None, {"light_max": 1, "chunk": 64, "heavy_blocks_per_cu": 1},
                                    {"light_max": 6, "chunk": 1024, "lepton_blocks_per_cu": 2,
                                     "photon_blocks_per_cu": 1},
                                    {"light_max": 0, "prepass_finish": 1, "prepass_blocks_per_cu": 1},
                                    {"light_max": 0, "prepass_finish": 0, "chunk": 128},
                                    {"light_max": 6, "light_tile": 128, "bins_per_octave": 4,
                                     "scatter_blocks_per_cu": 1},
                                    {"light_max": 0, "bins_per_octave": 32, "scatter_blocks_per_cu": 16}])
def test_binned_equals_naive_c2(tuning):
    from paper_2008_10468_amd import qed
    w = workloads.c2(n_e=20000, n_g=5000, seed=3)
    a, sa = _run(w, qed.QED_SCHED_NAIVE, fields_fn=workloads.c2_field)
    b, sb = _run(w, qed.QED_SCHED_BINNED, tuning=tuning, fields_fn=workloads.c2_field)
    for s in range(3):
        assert a[s]["id"].size == b[s]["id"].size
        for k in ("id", "ux", "uy", "uz", "x", "y", "z", "w"):
            assert np.array_equal(a[s][k], b[s][k]), (s, k)
    assert list(sa.substeps) == list(sb.substeps) and sa.emissions == sb.emissions


@pytest.mark.parametrize("slots", [64, 128, 256])
def test_tiled_equals_naive_c2(slots):
    """The tile-sorted scheduler at each tile size gives the naive kernel's results bit for bit."""
    from paper_2008_10468_amd import qed
    w = workloads.c2(n_e=20000, n_g=5000, seed=4)
    a, sa = _run(w, qed.QED_SCHED_NAIVE, fields_fn=workloads.c2_field)
    b, sb = _run(w, qed.QED_SCHED_TILED, tuning={"tiled_slots": slots}, fields_fn=workloads.c2_field)
    for s in range(3):
        for k in ("id", "ux", "uy", "uz", "x", "y", "z", "w"):
            assert np.array_equal(a[s][k], b[s][k]), (slots, s, k)
    assert list(sa.substeps) == list(sb.substeps) and sa.emissions == sb.emissions


@pytest.mark.parametrize("key", ["c3/binned", "c5/binned", "c5r/binned", "w5/binned", "w5r/binned"])
def test_recorded_tuning_binned_equals_naive(key):
    """The launch shapes and scheduler parameters the autotuner recorded for the hot spot
    (plain: c3; optical-depth path with the shipped network: c5, with rejection energies:
    c5r) and for the weak uniform field (w5, w5r) give the naive scheduler's results bit
    for bit on 2^15 electrons over two steps (c5, w5: the heavy queue's two-group network
    passes against the naive pass's single-group ones)."""
    import json
    import os
    from paper_2008_10468_amd import qed
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    tuning = json.load(open(os.path.join(root, "paper_2008_10468_amd", "tuning_gfx950.json")))[key]["tuning"]
    surr = key.startswith(("c5", "w5"))
    net = key.startswith(("c5/", "w5/"))
    m = np.load(os.path.join(root, "paper_2008_10468_amd", "models", "sampler_gfx950.npz")) if net else None
    if key.startswith("w5"):
        w = workloads.weak(n=1 << 15, seed=13)
    else:
        w = workloads.c3(n=1 << 15, hot_fraction=0.2, seed=12)
    zero = {k: np.zeros(1) for k in ("ex", "ey", "ez", "bx", "by", "bz")}
    res = []
    for sched, tu in ((qed.QED_SCHED_NAIVE, None), (qed.QED_SCHED_BINNED, tuning)):
        g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 15, 16, 1 << 19), pairs=False,
                          scheduler=sched, sampler=qed.QED_SAMPLER_SURROGATE if surr else qed.QED_SAMPLER_REJECTION)
        if net:
            assert qed.qed_sampler_set(g.ctx, m["params"], m["fallback"], float(m["log10_chi_lo"]),
                                       float(m["log10_chi_hi"])) == qed.QED_OK
        if tu:
            t = qed.qed_get_tuning(g.ctx)
            for k, v in tu.items():
                setattr(t, k, int(v))
            assert qed.qed_set_tuning(g.ctx, t) == qed.QED_OK
        g.load_state(w)
        g.set_fields(None, per_species=[w["fields"], zero, zero])
        for step in range(2):
            g.step(w["dt"], 7, step)
            assert g.sync()[0] == qed.QED_OK
        res.append(([_sorted(g.sp[k].download()) for k in (0, 2)], g.stats()))
        g.close()
    (a, sa), (b, sb) = res
    for s in range(2):
        for k in a[s]:
            assert np.array_equal(a[s][k], b[s][k]), (key, s, k)
    assert list(sa.substeps) == list(sb.substeps) and sa.emissions == sb.emissions and sa.emissions > 1000
    assert sb.heavy_particles > 0


def test_binned_hot_spot_matches_oracle():
    """C3 recipe in miniature: 30% hot, per-particle fields, binned scheduler."""
    from paper_2008_10468_amd import qed
    w = workloads.c3(n=8000, hot_fraction=0.3, seed=9)
    zero = {k: np.zeros(1) for k in ("ex", "ey", "ez", "bx", "by", "bz")}
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(8000, 16, 1 << 18), pairs=False,
                      scheduler=qed.QED_SCHED_BINNED)
    g.load_state(w)
    g.set_fields(None, per_species=[w["fields"], zero, zero])
    before = g.sp[0].download()
    g.step(w["dt"], 2, 0)
    assert g.sync()[0] == qed.QED_OK
    ev = g.sp[0].events_host(8000)
    after = g.sp[0].download()
    fh = as_precision(w["fields"], qed.QED_PREC_MIXED)
    ost = {k: before[k].copy() for k in ("x", "y", "z", "ux", "uy", "uz", "w", "id")}
    ch, nsub, nev, _ = oracle.lepton_step(ost, fh, -1.0, w["dt"], 2, 0, rng_bits=24)
    assert np.mean(nev == ev) >= 0.9999
    assert nsub.max() > 100           # the hot spot really is heavy
    same = nev == ev
    du = np.linalg.norm(np.stack([after[k] - ost[k] for k in ("ux", "uy", "uz")]), axis=0)
    um = np.linalg.norm(np.stack([ost[k] for k in ("ux", "uy", "uz")]), axis=0)
    assert np.all((du / um)[same] <= 2e-5 + 2e-7 * nsub[same])
    g.close()


def test_binned_fp64_c1_identical_events():
    from paper_2008_10468_amd import qed
    w = workloads.c1(n=2000)
    g = qed.Generator(precision=qed.QED_PREC_F64, capacity=(2048, 16, 1 << 16), pairs=False,
                      scheduler=qed.QED_SCHED_BINNED)
    g.load_state(w)
    g.set_fields(w["fields"])
    ost = {k: v.copy() for k, v in w["electrons"].items()}
    for s in range(3):
        g.step(w["dt"], 1, s)
        assert g.sync()[0] == qed.QED_OK
        ev = g.sp[0].events_host(2000)
        _, _, nev, _ = oracle.lepton_step(ost, w["fields"], -1.0, w["dt"], 1, s, rng_bits=53)
        assert np.array_equal(ev, nev)
    g.close()


def test_tuning_validation():
    from paper_2008_10468_amd import qed
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(16, 16, 16))
    t = qed.qed_get_tuning(g.ctx)
    t.chunk = 100      # not a multiple of 64
    assert qed.qed_set_tuning(g.ctx, t) == qed.QED_ERR_INVALID_ARG
    t.chunk = 128
    t.resolve_batch = 0       # 1..64
    assert qed.qed_set_tuning(g.ctx, t) == qed.QED_ERR_INVALID_ARG
    t.resolve_batch = 16
    t.prepass_finish = 2      # 0 or 1
    assert qed.qed_set_tuning(g.ctx, t) == qed.QED_ERR_INVALID_ARG
    t.prepass_finish = 1
    t.prepass_blocks_per_cu = 0
    assert qed.qed_set_tuning(g.ctx, t) == qed.QED_ERR_INVALID_ARG
    t.prepass_blocks_per_cu = 8
    t.light_max = 0           # no tile pass: the heavy queue takes every particle
    assert qed.qed_set_tuning(g.ctx, t) == qed.QED_OK
    t.light_max = 3
    assert qed.qed_set_tuning(g.ctx, t) == qed.QED_OK
    for field, bad, good in (("bins_per_octave", 3, 16), ("bins_per_octave", 33, 16), ("light_tile", 96, 512),
                             ("light_tile", 1024, 512), ("tiled_slots", 512, 256), ("tiled_slots", 0, 256),
                             ("scatter_blocks_per_cu", 0, 2)):
        setattr(t, field, bad)
        assert qed.qed_set_tuning(g.ctx, t) == qed.QED_ERR_INVALID_ARG, (field, bad)
        setattr(t, field, good)
        assert qed.qed_set_tuning(g.ctx, t) == qed.QED_OK
    g.close()

