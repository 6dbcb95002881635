"""GPU parity of in-step cascades (cascade_generations > 0) against the oracle.

Protocol: the GPU runs one step of the shower workload with G cascade passes;
the oracle's cascade_step runs the same step from the GPU's start-of-step state
with the same Philox streams.  Every particle of the end state is matched by its
deterministic id: the set of ids, positions, momenta, weights and the birth
times of the particles created in the step.  FP64 path: identical id sets (every
event decision agrees).  Mixed path: float rounding may flip a decision whose
test value lies within rounding of the acceptance probability, and every
descendant of such an event differs; so the mixed path is checked pass by pass,
each pass from the state the GPU reached before it (>= 99.99% agreement)."""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import RNG_BITS, as_precision

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("x", "y", "z", "ux", "uy", "uz", "w", "id")
CAP = (1 << 15, 1 << 15, 1 << 16)


def _gen(precision, gens, n=2048, scheduler=None, seed=6, capacity=CAP):
    from paper_2008_10468_amd import qed
    kw = {} if scheduler is None else {"scheduler": scheduler}
    g = qed.Generator(precision=precision, capacity=capacity, cascade_generations=gens, **kw)
    w = workloads.shower(n=n, seed=seed)
    g.load_state(w)
    g.set_fields(w["fields"])
    return g, w


def _run(g, w, seed=1, step=0):
    from paper_2008_10468_amd import qed
    before = [g.sp[s].download() for s in range(3)]
    print(f"cascade step: gens={g.cfg.cascade_generations} prec={g.precision} "
          f"n={[b['id'].size for b in before]}", flush=True)
    g.step(w["dt"], seed, step)
    st, rep = g.sync()
    assert st == qed.QED_OK, qed.status_string(st)
    after = [g.sp[s].download() for s in range(3)]
    return before, after


def _oracle(before, w, precision, gens, seed=1, step=0):
    strip = lambda d: {k: d[k].copy() for k in KEYS}
    f = as_precision(w["fields"], precision)
    ee, pp, gg, tl = oracle.cascade_step(strip(before[0]), strip(before[1]), strip(before[2]), f, w["dt"],
                                         seed, step, gens, p_max=w["p_max"], rng_bits=RNG_BITS[precision])
    return [ee, pp, gg], tl


def _match(gpu, orc):
    gi = {int(v): j for j, v in enumerate(gpu["id"])}
    oi = {int(v): j for j, v in enumerate(orc["id"])}
    common = sorted(set(gi) & set(oi))
    a = np.array([gi[k] for k in common], np.int64)
    b = np.array([oi[k] for k in common], np.int64)
    return a, b, len(set(gi) ^ set(oi)), len(oi)


def _compare(before, after, orc, dt, mom_rtol, pos_rtol, min_id_agree, min_close):
    out = []
    for s in range(3):
        a, b, diff, n_orc = _match(after[s], orc[s])
        assert after[s]["id"].size == np.unique(after[s]["id"]).size  # no id twice
        agree = 1.0 - diff / max(n_orc, 1)
        assert agree >= min_id_agree, (s, diff, n_orc)
        ug = np.stack([after[s][k][a] for k in ("ux", "uy", "uz")])
        uo = np.stack([orc[s][k][b] for k in ("ux", "uy", "uz")])
        du = np.linalg.norm(ug - uo, axis=0) / np.maximum(np.linalg.norm(uo, axis=0), 1.0)
        dx = np.max(np.abs(np.stack([after[s][k][a] - orc[s][k][b] for k in ("x", "y", "z")])), axis=0)
        close = (du <= mom_rtol) & (dx <= pos_rtol * dt + 1e-12 * np.abs(orc[s]["x"][b]))
        frac = float(np.mean(close)) if a.size else 1.0
        assert frac >= min_close, (s, frac, np.sort(du)[-5:], np.sort(dx)[-5:])
        assert np.array_equal(after[s]["w"][a], orc[s]["w"][b])
        # birth times of the particles created in the step
        new = ~np.isin(after[s]["id"][a], before[s]["id"])
        if new.any():
            bg = after[s]["birth"][a[new]]
            bo = orc[s]["birth"][b[new]]
            assert np.all((bo > 0) & (bo <= dt * (1 + 1e-12)))
            ok = np.abs(bg - bo) <= 1e-12 * dt
            assert float(np.mean(ok)) >= min_close, (s, float(np.mean(ok)))
        out.append((a.size, diff, int(new.sum())))
    return out


def test_fp64_cascade_matches_oracle():
    """Six cascade passes, FP64: the same particles, events and birth times."""
    from paper_2008_10468_amd import qed
    gens = 6
    g, w = _gen(qed.QED_PREC_F64, gens)
    before, after = _run(g, w)
    orc, tl = _oracle(before, w, qed.QED_PREC_F64, gens)
    # the workload really cascades: events in at least four passes
    deep = sum(1 for t in tl if t[0]["events"] + t[1]["events"] + t[2]["events"] > 0)
    assert deep >= 4, [(t[0]["events"], t[1]["events"]) for t in tl]
    res = _compare(before, after, orc, w["dt"], mom_rtol=1e-9, pos_rtol=1e-9, min_id_agree=1.0, min_close=1.0)
    assert all(r[2] > 0 for r in res), res
    st = g.stats()
    assert st.pairs == sum(t[0]["events"] for t in tl)
    assert st.emissions == sum(t[1]["events"] + t[2]["events"] for t in tl)
    g.close()


def _pass_check(inp, t0, out_gpu, new_gpu, w, precision, pass_no):
    """One pass from the state the GPU reached before it.  inp: the pass's particles
    per species (their state at the pass start), t0 their start times (None: 0);
    out_gpu: the GPU state after the pass; new_gpu: the particles the GPU created in
    the pass (per species, with birth times).  Returns the per-species agreement of
    the particles' outcomes (events and survival) and the children matched."""
    f = as_precision(w["fields"], precision)
    rb = RNG_BITS[precision]
    strip = lambda d: {k: np.ascontiguousarray(d[k]).copy() for k in KEYS}
    ge, pe, gg = strip(inp[0]), strip(inp[1]), strip(inp[2])
    chg, alive, gns, gnev, _ = oracle.photon_step(gg, f, w["dt"], 1, 0, p_max=w["p_max"], rng_bits=rb, t0=t0[2])
    che, ens, enev, _ = oracle.lepton_step(ge, f, -1.0, w["dt"], 1, 0, p_max=w["p_max"], rng_bits=rb, t0=t0[0])
    chp, pns, pnev, _ = oracle.lepton_step(pe, f, 1.0, w["dt"], 1, 0, p_max=w["p_max"], rng_bits=rb, t0=t0[1])
    orc_state = (ge, pe, gg)
    orc_nev = (enev, pnev, gnev)
    orc_nsub = (ens, pns, gns)
    agree = []
    for s in range(3):
        ids = orc_state[s]["id"]
        if ids.size == 0:
            agree.append(1.0)
            continue
        gi = {int(v): j for j, v in enumerate(out_gpu[s]["id"])}
        # events of each particle on the GPU: children it created in this pass
        par = np.concatenate([new_gpu[k]["parent"] for k in range(3)]) if s < 2 else \
            np.concatenate([new_gpu[k]["parent"] for k in range(2)])
        cnt = {}
        for v in par.tolist():
            cnt[v] = cnt.get(v, 0) + 1
        gnev_s = np.array([cnt.get(int(v), 0) for v in ids])
        same = gnev_s == orc_nev[s]
        if s == 2:   # photons: a decay creates two children, and the photon is gone
            present = np.array([int(v) in gi for v in ids])
            same = (gnev_s // 2 == orc_nev[s]) & (present == alive.astype(bool))
        agree.append(float(np.mean(same)))
        assert agree[-1] >= 0.9999, (pass_no, s, agree[-1], int((~same).sum()), ids.size)
        # survivors' momenta and positions (particles with the same events)
        keep = same & np.array([int(v) in gi for v in ids])
        a = np.array([gi[int(v)] for v in ids[keep]], np.int64)
        ug = np.stack([out_gpu[s][k][a] for k in ("ux", "uy", "uz")])
        uo = np.stack([orc_state[s][k][keep] for k in ("ux", "uy", "uz")])
        du = np.linalg.norm(ug - uo, axis=0) / np.maximum(np.linalg.norm(uo, axis=0), 1.0)
        tol = 2e-5 + 2e-7 * orc_nsub[s][keep]
        assert np.all(du <= tol), (pass_no, s, du.max())
    # the children, matched by id, with their birth times
    nmatch = 0
    tbmap = {}
    for s, (name, kinds) in enumerate((("e", [(chg, 1)]), ("p", [(chg, 2)]), ("g", [(che, 0), (chp, 0)]))):
        ids_o, tb_o = [], []
        for ch, kind in kinds:
            sel = ch["kind"] == kind
            ids_o.append(ch["id"][sel])
            tb_o.append(ch["tb"][sel])
        ids_o = np.concatenate(ids_o)
        tb_o = np.concatenate(tb_o)
        tbmap.update(zip(ids_o.tolist(), tb_o.tolist()))
        gi = {int(v): j for j, v in enumerate(new_gpu[s]["id"])}
        common = [j for j, v in enumerate(ids_o.tolist()) if v in gi]
        miss = ids_o.size + new_gpu[s]["id"].size - 2 * len(common)
        assert miss <= max(2, int(1e-4 * max(ids_o.size, 1)) * 2), (pass_no, s, miss, ids_o.size)
        if common:
            a = np.array([gi[int(ids_o[j])] for j in common])
            bg = new_gpu[s]["birth"][a]
            known = np.isfinite(bg)   # (the main pass's children: where a later run recorded it)
            assert np.all(np.abs(bg[known] - tb_o[common][known]) <= 1e-12 * w["dt"])
        nmatch += len(common)
    return agree, nmatch, tbmap


def test_mixed_cascade_each_pass_from_gpu_state():
    """Mixed precision, pass by pass: the GPU run with g follow-up passes gives the state
    that pass g + 1 starts from; the oracle runs that one pass from it (each particle
    from its birth time), and its result is compared with the GPU run with g + 1
    passes.  Float rounding in earlier passes then cannot compound: each pass's
    particles agree on their events and survival for >= 99.99%, and the children are
    matched by id with their birth times."""
    from paper_2008_10468_amd import qed
    gens = 4
    runs = []
    for g in range(gens + 1):
        gen, w = _gen(qed.QED_PREC_MIXED, g, n=3000)
        before, after = _run(gen, w)
        runs.append(after)
        gen.close()
    start = before
    known = [set(start[s]["id"].tolist()) for s in range(3)]
    # main pass: from the start state
    new0 = [{k: v[~np.isin(runs[0][s]["id"], start[s]["id"])] for k, v in runs[0][s].items()} for s in range(3)]
    # birth times of the main pass's children: a run with cascades records them
    b1 = [dict(zip(runs[1][s]["id"].tolist(), runs[1][s]["birth"].tolist())) for s in range(3)]
    for s in range(3):
        new0[s]["birth"] = np.array([b1[s].get(int(v), np.nan) for v in new0[s]["id"]])
    agree, m, tb0 = _pass_check(start, (None, None, None), runs[0], new0, w, qed.QED_PREC_MIXED, 0)
    print("pass 0 agreement", agree, "children matched", m, flush=True)
    total = m
    for g in range(gens):
        prev_known = [known[s] | set(runs[g - 1][s]["id"].tolist()) if g >= 1 else known[s] for s in range(3)]
        inp = [{k: v[~np.isin(runs[g][s]["id"], np.array(sorted(prev_known[s]), np.uint64))]
                for k, v in runs[g][s].items()} for s in range(3)]
        if g == 0:   # the main pass's children start at the birth times matched above
            for s in range(3):
                inp[s]["birth"] = np.array([tb0.get(int(v), np.nan) for v in inp[s]["id"]])
        assert all(np.all(np.isfinite(inp[s]["birth"])) for s in range(3))
        t0 = tuple(np.ascontiguousarray(inp[s]["birth"]) for s in range(3))
        done = [prev_known[s] | set(inp[s]["id"].tolist()) for s in range(3)]
        newg = [{k: v[~np.isin(runs[g + 1][s]["id"], np.array(sorted(done[s]), np.uint64))]
                 for k, v in runs[g + 1][s].items()} for s in range(3)]
        agree, m, _ = _pass_check(inp, t0, runs[g + 1], newg, w, qed.QED_PREC_MIXED, g + 1)
        print("pass", g + 1, "particles", [inp[s]["id"].size for s in range(3)], "agreement", agree,
              "children matched", m, flush=True)
        total += m
    assert total > 1000


@pytest.mark.parametrize("precision", ["F64", "MIXED"])
def test_cascade_schedulers_agree(precision):
    """The main pass may run on any scheduler; the end state is the same bit for bit."""
    from paper_2008_10468_amd import qed
    prec = getattr(qed, "QED_PREC_" + precision)
    res = []
    for sched in (qed.QED_SCHED_NAIVE, qed.QED_SCHED_BINNED, qed.QED_SCHED_TILED):
        g, w = _gen(prec, 3, scheduler=sched)
        _, after = _run(g, w)
        order = [np.argsort(a["id"]) for a in after]
        res.append([{k: a[k][o] for k in KEYS + ("birth",)} for a, o in zip(after, order)])
        g.close()
    for other in res[1:]:
        for s in range(3):
            for k in KEYS:
                assert np.array_equal(res[0][s][k], other[s][k]), (s, k)
            new = ~np.isin(res[0][s]["id"], np.arange(3 * 2048, dtype=np.uint64))
            assert np.array_equal(res[0][s]["birth"][new], other[s]["birth"][new])


def test_main_pass_is_the_plain_step():
    """Cascade passes touch only the particles created in the step: the particles present
    at the start end exactly as in a step without cascades, and the same photons decay."""
    from paper_2008_10468_amd import qed
    g3, w = _gen(qed.QED_PREC_MIXED, 3)
    before, a3 = _run(g3, w)
    g3.close()
    g0 = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=CAP)
    g0.load_state(w)
    g0.set_fields(w["fields"])
    _, a0 = _run(g0, w)
    g0.close()
    for s in range(3):
        old = before[s]["id"]
        k3 = np.isin(a3[s]["id"], old)
        k0 = np.isin(a0[s]["id"], old)
        o3 = np.argsort(a3[s]["id"][k3])
        o0 = np.argsort(a0[s]["id"][k0])
        for k in KEYS:
            assert np.array_equal(a3[s][k][k3][o3], a0[s][k][k0][o0]), (s, k)
    # without cascades the children carry no birth array and have not moved
    assert a0[2]["id"].size < a3[2]["id"].size or a0[0]["id"].size < a3[0]["id"].size


def test_cascade_capacity_overflow_is_reported():
    from paper_2008_10468_amd import qed
    g, w = _gen(qed.QED_PREC_MIXED, 4, n=2048, capacity=(2300, 2300, 1 << 16))
    g.step(w["dt"], 1, 0)
    st, rep = g.sync()
    assert st == qed.QED_ERR_CAPACITY
    assert rep.required_capacity[0] > 2300 or rep.required_capacity[1] > 2300
    g.close()


def test_cascade_bad_configuration():
    from paper_2008_10468_amd import qed
    for gens, sampler in ((65, qed.QED_SAMPLER_REJECTION), (1, qed.QED_SAMPLER_SURROGATE)):
        cfg = qed.qed_config_default()
        cfg.cascade_generations = gens
        cfg.sampler = sampler
        ctx = C.c_void_p()
        assert qed.load().qed_init(C.byref(ctx), C.byref(cfg)) == qed.QED_ERR_INVALID_ARG
    g, w = _gen(qed.QED_PREC_MIXED, 2, n=64)
    p = g.particles()
    p.photons.birth = None
    flds = [f.struct() for f in g.fields]
    assert qed.qed_step(g.ctx, p, flds, w["dt"], 1, 0) == qed.QED_ERR_INVALID_ARG
    # per-slot fields: the library has no field for a new slot
    per_slot = {k: np.full(64, v[0]) for k, v in w["fields"].items()}
    g.set_fields(per_slot)
    assert qed.qed_step(g.ctx, g.particles(), [f.struct() for f in g.fields], w["dt"], 1, 0) == \
        qed.QED_ERR_INVALID_ARG
    g.close()
