"""Autotuner for the generator's launch shapes and scheduler parameters.

The per-particle cost of the generator is very uneven (a particle's sub-step
count N ranges from 1 to about 1000 in a hot spot), so the best launch shape
depends on the workload: blocks per compute unit of each kernel, the largest N
handled by the light pass of the binned scheduler, and the number of queue
entries a wave claims at a time in its persistent heavy pass.

The surrogate path adds the number of emissions a wave lets wait before
resolving them together; the binned scheduler whether its pre-pass finishes
particles of one quiet sub-step, the grid of its placement pass, the number of
sub-step-count bins per octave (how close the counts in one wave of the heavy
queue are) and the tile of its light pass; the tile-sorted scheduler its tile.

`tune` measures candidate settings on the real workload and device with
coordinate descent: starting from the library's defaults, it sweeps one
parameter at a time over its candidate values, keeps the fastest, and repeats
the sweep.  Each candidate is timed as a HIP graph of `steps` whole steps from
the same initial state (best of `repeats` replays).  Every setting must give
the same device counters (sub-steps, events) as the defaults: the generator's
results do not depend on the launch shape, and a candidate that changes them is
rejected loudly.

The table written by `main` maps "<workload>/<scheduler>" to the chosen
setting with its measured time; the benchmark applies it.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys

from . import qed

SPACE = {
    "lepton_blocks_per_cu": (1, 2, 4, 8, 16, 32, 64, 128, 256),
    "photon_blocks_per_cu": (1, 2, 4, 8, 16, 32, 64, 128),
    "heavy_blocks_per_cu": (1, 2, 3, 4, 8, 16),
    "light_max": (0, 1, 2, 4, 8, 16, 32, 48, 64, 128, 256),
    "chunk": (64, 128, 256, 512, 1024, 4096),
    "resolve_batch": (4, 8, 12, 16, 24, 32, 48, 64),
    "prepass_blocks_per_cu": (4, 8, 16, 32, 64, 128, 256, 512),
    "prepass_finish": (0, 1),
    "scatter_blocks_per_cu": (1, 2, 4, 8, 16),
    "bins_per_octave": (4, 8, 16, 32),
    "light_tile": (128, 256, 512),
    "tiled_slots": (64, 128, 256),
}
NAIVE_KEYS = ("lepton_blocks_per_cu", "photon_blocks_per_cu")
MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models", "sampler_gfx950.npz")
BINNED_KEYS = ("lepton_blocks_per_cu", "photon_blocks_per_cu", "heavy_blocks_per_cu", "light_max", "chunk",
               "prepass_blocks_per_cu", "prepass_finish", "scatter_blocks_per_cu", "bins_per_octave", "light_tile")
TILED_KEYS = ("lepton_blocks_per_cu", "photon_blocks_per_cu", "tiled_slots")
SURROGATE_KEYS = ("resolve_batch",)   # added for workloads on the lepton optical-depth path


def _settings(g):
    t = qed.qed_get_tuning(g.ctx)
    return {k: int(getattr(t, k)) for k in SPACE}


def _apply(g, setting):
    t = qed.qed_get_tuning(g.ctx)
    for k, v in setting.items():
        setattr(t, k, int(v))
    st = qed.qed_set_tuning(g.ctx, t)
    if st != qed.QED_OK:
        raise qed.QedError(st, f"qed_set_tuning {setting}")


def time_setting(torch, g, stream, setting, state, fields_for_step, dt, seed, steps, repeats=2):
    """Milliseconds for `steps` graph-captured steps from `state`, and the counters."""
    lib = qed.load()
    _apply(g, setting)
    parts = C.byref(g.particles())
    flds = [fields_for_step(s) for s in range(steps)]

    def enqueue():
        for s in range(steps):
            st = lib.qed_step(g.ctx, parts, flds[s], float(dt), int(seed), s)
            if st != qed.QED_OK:
                raise qed.QedError(st, "qed_step")

    # one eager pass warms up and sizes the library's scratch before capture
    g.load_state(state)
    enqueue()
    st, rep = g.sync()
    if st != qed.QED_OK:
        raise qed.QedError(st, "qed_sync")
    assert qed.qed_graph_begin(g.ctx) == qed.QED_OK
    enqueue()
    st, graph = qed.qed_graph_end(g.ctx)
    if st != qed.QED_OK:
        raise qed.QedError(st, "qed_graph_end")
    best, counters = None, None
    try:
        for _ in range(repeats):
            g.load_state(state)
            qed.qed_reset_stats(g.ctx)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            assert qed.qed_graph_launch(g.ctx, graph) == qed.QED_OK
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            st, rep = g.sync()
            if st != qed.QED_OK:
                raise qed.QedError(st, "qed_sync")
            s = g.stats()
            c = (tuple(s.substeps), s.emissions, s.pairs, tuple(rep.n))
            if counters is not None and c != counters:
                raise RuntimeError(f"replays of one setting disagree: {c} vs {counters}")
            counters = c
            best = ms if best is None else min(best, ms)
    finally:
        qed.qed_graph_destroy(graph)
    return best, counters


def tune(torch, g, stream, state, fields_for_step, dt, seed, steps, keys, passes=2, log=print):
    """Coordinate descent over SPACE[keys]; returns (setting, ms, history)."""
    cur = _settings(g)
    ms0, ref = time_setting(torch, g, stream, cur, state, fields_for_step, dt, seed, steps)
    best_ms = ms0
    history = [{"setting": dict(cur), "ms": ms0}]
    log(f"autotune: defaults {cur}: {ms0:.3f} ms")
    for p in range(passes):
        changed = False
        for k in keys:
            for v in SPACE[k]:
                if v == cur[k]:
                    continue
                cand = dict(cur, **{k: v})
                try:
                    ms, c = time_setting(torch, g, stream, cand, state, fields_for_step, dt, seed, steps)
                except qed.QedError as e:      # e.g. a combination the library rejects
                    log(f"autotune: {cand} rejected: {e}")
                    continue
                if c != ref:
                    raise RuntimeError(f"setting {cand} changed the results: {c} vs {ref}")
                history.append({"setting": cand, "ms": ms})
                log(f"autotune: pass {p} {k}={v}: {ms:.3f} ms")
                if ms < best_ms * 0.99:      # demand a clear gain, not noise
                    best_ms, cur, changed = ms, cand, True
        if not changed:
            break
    _apply(g, cur)
    return cur, best_ms, ms0, history


def _workload(name, torch, workloads, sched, stream, steps):
    """Generator, state, per-step fields, dt and seed of a named workload."""
    if name in ("c2", "c2s"):
        # c2s: the same population on both optical-depth paths, with the shipped network
        import numpy as np
        w = workloads.c2()
        sur = qed.QED_SAMPLER_SURROGATE if name == "c2s" else qed.QED_SAMPLER_REJECTION
        g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 23, 1 << 23, 1 << 25),
                          parent=False, events=False, scheduler=sched, stream=stream.cuda_stream,
                          sampler=sur, pair_sampler=sur)
        if name == "c2s":
            m = np.load(MODEL)
            st = qed.qed_sampler_set(g.ctx, m["params"], m["fallback"], float(m["log10_chi_lo"]),
                                     float(m["log10_chi_hi"]))
            if st != qed.QED_OK:
                raise qed.QedError(st, "qed_sampler_set")
        E = np.array([[workloads.c2_field(s)[k][0] for k in ("ex", "ey", "ez", "bx", "by", "bz")]
                      for s in range(steps)], np.float64)
        table = [torch.from_numpy(E[:, j].copy()).to(torch.float32).cuda() for j in range(6)]

        def fields(s):
            f = qed.qed_field()
            for j, k in enumerate(("ex", "ey", "ez", "bx", "by", "bz")):
                setattr(f, k, table[j].data_ptr() + 4 * s)
            f.stride = 0
            return (qed.qed_field * 3)(f, f, f)
        g._keep = table
        return g, w, fields
    if name == "c3":
        w = workloads.c3()
        n = w["electrons"]["id"].size
        g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, 16, int(0.65 * n * steps) + (1 << 23)),
                          pairs=False, parent=False, events=False, scheduler=sched,
                          stream=stream.cuda_stream)
        zero = workloads.uniform_field()
        g.set_fields(None, per_species=[w["fields"], zero, zero])
        fl = [f.struct() for f in g.fields]
        return g, w, lambda s: (qed.qed_field * 3)(*fl)
    if name in ("c5", "c5r", "w5", "w5r"):
        # the hot-spot workload (c5) or the weak uniform field (w5) on the surrogate path,
        # with the network shipped for gfx950 or with rejection energies (c5r, w5r)
        import numpy as np
        w = workloads.c3() if name.startswith("c") else workloads.weak()
        n = w["electrons"]["id"].size
        per = 0.65 if name.startswith("c") else 1.0   # photons per electron and step, about
        g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, 16, int(per * n * steps) + (1 << 23)),
                          pairs=False, parent=False, events=False, scheduler=sched,
                          stream=stream.cuda_stream, sampler=qed.QED_SAMPLER_SURROGATE)
        if name in ("c5", "w5"):
            m = np.load(MODEL)
            st = qed.qed_sampler_set(g.ctx, m["params"], m["fallback"], float(m["log10_chi_lo"]),
                                     float(m["log10_chi_hi"]))
            if st != qed.QED_OK:
                raise qed.QedError(st, "qed_sampler_set")
        zero = workloads.uniform_field()
        g.set_fields(None, per_species=[w["fields"], zero, zero])
        fl = [f.struct() for f in g.fields]
        return g, w, lambda s: (qed.qed_field * 3)(*fl)
    raise ValueError(name)


def main(argv=None):
    ap = argparse.ArgumentParser(description="Tune launch shapes of the QED generator on this GPU")
    ap.add_argument("--workload", choices=("c2", "c2s", "c3", "c5", "c5r", "w5", "w5r"), action="append")
    ap.add_argument("--scheduler", choices=("naive", "binned", "tiled"), action="append")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import torch
    import workloads

    torch.cuda.set_device(0)
    table = json.load(open(args.out)) if os.path.exists(args.out) else {}
    table["device"] = torch.cuda.get_device_properties(0).gcnArchName
    for wl in args.workload or ["c2"]:
        for sn in args.scheduler or ["naive", "binned", "tiled"]:
            sched = {"naive": qed.QED_SCHED_NAIVE, "binned": qed.QED_SCHED_BINNED, "tiled": qed.QED_SCHED_TILED}[sn]
            stream = torch.cuda.Stream()
            g, w, fields = _workload(wl, torch, workloads, sched, stream, args.steps)
            keys = {"binned": BINNED_KEYS, "tiled": TILED_KEYS}.get(sn, NAIVE_KEYS)
            if wl in ("c2s", "c5", "c5r", "w5", "w5r"):
                keys = keys + SURROGATE_KEYS
            best, ms, ms0, hist = tune(torch, g, stream, w, fields, w["dt"], w["seed"], args.steps, keys,
                                       passes=args.passes, log=lambda *a: print(*a, flush=True))
            table[f"{wl}/{sn}"] = {"tuning": best, "ms_per_step": ms / args.steps,
                                   "default_ms_per_step": ms0 / args.steps, "steps": args.steps,
                                   "candidates": len(hist)}
            print(f"autotune: {wl}/{sn}: {best} {ms / args.steps:.4f} ms/step "
                  f"(defaults {ms0 / args.steps:.4f})", flush=True)
            g.close()
            with open(args.out, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
