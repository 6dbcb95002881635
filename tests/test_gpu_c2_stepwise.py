"""C2 at full size over its 200 steps (1,048,576 electrons + 262,144 photons in the
rotating E field, mixed precision, the benchmark's launch shapes), checked against
the oracle in two ways:

* step by step: at steps 10, 50, 100 and 199 the GPU's state at the step's start is
  the oracle's input for that one step, on a sample of 2^16 particles drawn from
  every part of the grown population (original electrons, electrons and positrons
  from pairs, original photons, emitted photons).  Each sampled particle's events
  (emissions; decays of photons) are identical on >= 99.99% of them, survivors'
  momenta agree to float accuracy, and their children are matched by id.
* over the whole run: a subset of the initial population (2^14 electrons and 2^12
  photons) runs all 200 steps on the GPU and, independently, in the oracle; the
  pair yield and the photon spectrum (20 bins of log10 energy) agree within 3 sigma.

Trajectories in float and double drift apart over many steps (and N can change
between them), so the per-particle comparison is made step-wise from GPU snapshots;
the whole-run comparison is statistical."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import as_precision

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECK_STEPS = (10, 50, 100, 199)


def _gen(qed, capacity):
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=capacity)
    t = qed.qed_get_tuning(g.ctx)
    for k, v in json.load(open(os.path.join(ROOT, "paper_2008_10468_amd", "tuning_gfx950.json")))["c2/naive"][
            "tuning"].items():
        setattr(t, k, int(v))
    assert qed.qed_set_tuning(g.ctx, t) == qed.QED_OK
    return g


def _mom(d, idx=None):
    m = np.stack([d["ux"], d["uy"], d["uz"]])
    return m if idx is None else m[:, idx]


def _sample(before, n_e0, n_g0, rng):
    """2^16 slots over the populations: e- originals / from pairs, e+, photons original / emitted."""
    e_ids, g_ids = before[0]["id"], before[2]["id"]
    e_orig = np.flatnonzero(e_ids < n_e0)            # pair electrons carry hashed ids
    e_new = np.flatnonzero(e_ids >= n_e0)
    g_orig = np.flatnonzero((g_ids >= n_e0) & (g_ids < n_e0 + n_g0))
    g_new = np.setdiff1d(np.arange(g_ids.size), g_orig)
    take = lambda a, k: np.sort(rng.choice(a, min(k, a.size), replace=False)) if a.size else a
    se = np.sort(np.concatenate([take(e_orig, 24576), take(e_new, 4096)]))
    sp = take(np.arange(before[1]["id"].size), 4096)
    sg = np.sort(np.concatenate([take(g_orig, 16384), take(g_new, 16384)]))
    return se, sp, sg


def _sub(d, idx):
    return {k: np.ascontiguousarray(d[k][idx]) for k in ("x", "y", "z", "ux", "uy", "uz", "w", "id")}


def _children_check(gpu_after, n0, orc_ch, kind, parents, tol):
    """Children of the sampled parents: ids present on the GPU (appended after n0), momenta."""
    sel = (orc_ch["kind"] == kind) & np.isin(orc_ch["parent"], parents)
    ids = orc_ch["id"][sel]
    gi = {int(v): j for j, v in enumerate(gpu_after["id"][n0:].tolist())} if kind != 0 else \
        {int(v): j for j, v in enumerate(gpu_after["id"].tolist())}
    found = np.array([int(v) in gi for v in ids])
    if ids.size:
        j = np.array([gi[int(v)] for v in ids[found]], np.int64) + (n0 if kind != 0 else 0)
        pg = _mom(gpu_after, j)
        po = np.stack([orc_ch["px"][sel][found], orc_ch["py"][sel][found], orc_ch["pz"][sel][found]])
        d = np.linalg.norm(pg - po, axis=0) / np.maximum(np.linalg.norm(po, axis=0), 1e-30)
        assert d.size == 0 or d.max() <= tol, d.max()
    return int(found.sum()), int((~found).sum())


def test_c2_full_size_stepwise_from_gpu_snapshots():
    from paper_2008_10468_amd import qed
    w = workloads.c2()
    n_e0, n_g0 = w["electrons"]["id"].size, w["photons"]["id"].size
    g = _gen(qed, (1 << 23, 1 << 22, 1 << 25))
    g.load_state(w)
    g.set_fields(workloads.c2_field(0))
    rng = np.random.default_rng(199)
    checked = []
    for step in range(200):
        for f in g.fields:
            f.set_uniform(workloads.c2_field(step))
        if step not in CHECK_STEPS:
            g.step(w["dt"], w["seed"], step)
            continue
        before = [g.sp[s].download() for s in range(3)]
        n0 = [b["id"].size for b in before]
        print("C2 stepwise: step", step, "population", n0, flush=True)
        g.step(w["dt"], w["seed"], step)
        st, rep = g.sync()
        assert st == qed.QED_OK, qed.status_string(st)
        after = [g.sp[s].download() for s in range(3)]
        events = [g.sp[s].events_host(n0[s]) for s in range(3)]
        se, sp, sg = _sample(before, n_e0, n_g0, rng)
        fh = as_precision(workloads.c2_field(step), qed.QED_PREC_MIXED)
        out = {}
        for s, idx, q in ((0, se, -1.0), (1, sp, 1.0)):
            sub = _sub(before[s], idx)
            och, nsub, nev, _ = oracle.lepton_step(sub, fh, q, w["dt"], w["seed"], step, rng_bits=24)
            same = nev == events[s][idx]
            out[s] = (float(np.mean(same)) if idx.size else 1.0, idx.size)
            assert not idx.size or np.mean(same) >= 0.9999, (step, s, np.mean(same))
            du = np.linalg.norm(_mom(after[s], idx) - _mom(sub), axis=0) / np.maximum(
                np.linalg.norm(_mom(sub), axis=0), 1.0)
            assert np.all(du[same] <= 2e-5 + 2e-7 * nsub[same]), (step, s, du[same].max())
            found, miss = _children_check(after[2], 0, och, 0, sub["id"][same], 2e-5 + 2e-7 * int(nsub.max()))
            assert miss == 0, (step, s, miss)
        sub = _sub(before[2], sg)
        pch, alive, _, pnev, _ = oracle.photon_step(sub, fh, w["dt"], w["seed"], step, rng_bits=24)
        same = pnev == events[2][sg]
        out[2] = (float(np.mean(same)), sg.size)
        assert np.mean(same) >= 0.9999, (step, np.mean(same))
        ids_g = set(after[2]["id"].tolist())
        surv = np.array([int(v) in ids_g for v in sub["id"]])
        assert np.mean(surv == alive.astype(bool)) >= 0.9999
        for s, kind in ((0, 1), (1, 2)):
            found, miss = _children_check(after[s], n0[s], pch, kind, sub["id"][same], 2e-5)
            assert miss == 0, (step, kind, miss)
        print("C2 stepwise: step", step, "agreement e-/e+/photons", out, flush=True)
        checked.append(step)
    assert checked == list(CHECK_STEPS)
    st = g.stats()
    assert st.pairs > 1000 and st.emissions > 1e6
    g.close()


def _oracle_run(e, p, ph, steps, dt, seed):
    """The oracle on its own for `steps` steps: appends, photon removal (as the generator)."""
    keys = ("x", "y", "z", "ux", "uy", "uz", "w", "id")
    sp = {"e": e, "p": p, "g": ph}

    def append(dst, ch, sel):
        for k, ck in zip(keys, ("x", "y", "z", "px", "py", "pz", "w", "id")):
            dst[k] = np.concatenate([dst[k], ch[ck][sel]])
    pairs = 0
    for step in range(steps):
        f = as_precision(workloads.c2_field(step), 1)
        chg, alive, _, _, tg = oracle.photon_step(sp["g"], f, dt, seed, step, rng_bits=24)
        che, _, _, _ = oracle.lepton_step(sp["e"], f, -1.0, dt, seed, step, rng_bits=24)
        chp, _, _, _ = oracle.lepton_step(sp["p"], f, 1.0, dt, seed, step, rng_bits=24)
        sp["g"] = {k: v[alive.astype(bool)] for k, v in sp["g"].items()}
        append(sp["e"], chg, chg["kind"] == 1)
        append(sp["p"], chg, chg["kind"] == 2)
        append(sp["g"], che, slice(None))
        append(sp["g"], chp, slice(None))
        pairs += int(tg["events"])
    return sp, pairs


def test_c2_full_run_spectrum_and_pair_yield():
    from paper_2008_10468_amd import qed
    w = workloads.c2()
    rng = np.random.default_rng(7)
    ie = np.sort(rng.choice(w["electrons"]["id"].size, 1 << 14, replace=False))
    ig = np.sort(rng.choice(w["photons"]["id"].size, 1 << 12, replace=False))
    sub = {"electrons": workloads.subset(w["electrons"], ie), "positrons": w["positrons"],
           "photons": workloads.subset(w["photons"], ig)}
    for s in sub.values():
        for k in ("ux", "uy", "uz", "w"):
            s[k] = s[k].astype(np.float32).astype(np.float64)
    g = _gen(qed, (1 << 17, 1 << 15, 1 << 20))
    g.load_state(sub)
    g.set_fields(workloads.c2_field(0))
    for step in range(200):
        for f in g.fields:
            f.set_uniform(workloads.c2_field(step))
        g.step(w["dt"], w["seed"], step)
    st, rep = g.sync()
    assert st == qed.QED_OK
    gpu = [g.sp[s].download() for s in range(3)]
    gpu_pairs = g.stats().pairs
    g.close()
    print("C2 full run: GPU done, oracle running", flush=True)
    orc, orc_pairs = _oracle_run({k: v.copy() for k, v in sub["electrons"].items()},
                                 {k: v.copy() for k, v in sub["positrons"].items()},
                                 {k: v.copy() for k, v in sub["photons"].items()}, 200, w["dt"], w["seed"])
    print("C2 full run: pairs GPU", gpu_pairs, "oracle", orc_pairs, "photons", gpu[2]["id"].size,
          orc["g"]["id"].size, flush=True)
    assert orc_pairs > 50
    assert abs(gpu_pairs - orc_pairs) <= 3.0 * math.sqrt(gpu_pairs + orc_pairs) + 1
    eg = np.linalg.norm(_mom(gpu[2]), axis=0)
    eo = np.linalg.norm(np.stack([orc["g"]["ux"], orc["g"]["uy"], orc["g"]["uz"]]), axis=0)
    edges = np.linspace(-2.0, 5.5, 21)
    hg, _ = np.histogram(np.log10(np.maximum(eg, 1e-30)), edges)
    ho, _ = np.histogram(np.log10(np.maximum(eo, 1e-30)), edges)
    sig = np.sqrt(hg + ho) + 1.0
    assert np.all(np.abs(hg - ho) <= 3.0 * sig), np.stack([hg, ho])
    assert hg.sum() > 10000
