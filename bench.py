#!/usr/bin/env python3
"""Throughput of the QED event generator on one MI355X.

A step is one global QED-PIC step of the whole generator (Algorithm 2 on all
photons, Algorithm 1 on all electrons and positrons, appends, photon compaction)
over the default workload: 1,048,576 electrons + 262,144 photons in a uniform E
field of 1e-3 Schwinger units rotating with period 200 steps, mixed precision,
buffers growing by appends for all timed steps.  Metric: particle-sub-steps per
second (sub-steps of the adaptive generator summed over all particles), with
events per second beside it.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (packed) peak
FP64_VECTOR_PEAK_TFLOPS = 78.6

# Algorithmic work per unit, counted from the kernel source (mixed precision).
# Floating-point operations: FMA = 2, each reciprocal / square root / cube root /
# exponential = 1.  HBM bytes: the arrays a kernel must touch for one particle.
FLOPS_PER_LEPTON_SUBSTEP = 170      # Boris push 52, gamma and move 15, chi 40, candidate 14,
                                    # F and G 37, acceptance 12
FLOPS_PER_PHOTON_SUBSTEP = 62       # move 6, candidate 6, F and G 37, acceptance 13
BYTES_PER_LEPTON_STEP = 80          # read u 12 + id 8 + position 24; write u 12 + position 24
BYTES_PER_EMISSION = 52             # weight read 4; position 24 + k 12 + weight 4 + id 8 written
BYTES_PER_PHOTON_STEP = 61          # read k 12 + position 24; write position 24 + flag 1
BYTES_PER_BINNED_EXTRA = 8          # sub-step count read 4 + queue entry read 4 (heavy pass)
def log(*a):
    print(*a, file=sys.stderr, flush=True)


def c2_setup(torch, qed, workloads, steps_total, sched, stream=None):
    w = workloads.c2()
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 23, 1 << 23, 1 << 25),
                      parent=False, events=False, scheduler=sched,
                      stream=None if stream is None else stream.cuda_stream)
    # one frozen field per global step, resident on the device: step s reads entry s
    E = np.array([[workloads.c2_field(s)[k][0] for k in ("ex", "ey", "ez", "bx", "by", "bz")]
                  for s in range(steps_total)], np.float64)
    table = [torch.from_numpy(E[:, j].copy()).to(torch.float32).cuda() for j in range(6)]

    def field(s):
        f = qed.qed_field()
        for j, k in enumerate(("ex", "ey", "ez", "bx", "by", "bz")):
            setattr(f, k, table[j].data_ptr() + 4 * s)
        f.stride = 0
        return f
    return w, g, field


def run_steps(qed, g, field, w, first, count):
    """Enqueue count steps; ABI structs are built before the loop."""
    import ctypes as C
    lib = qed.load()
    parts = C.byref(g.particles())
    flds = [(qed.qed_field * 3)(field(s), field(s), field(s)) for s in range(first, first + count)]
    dt, seed = float(w["dt"]), int(w["seed"])
    for j, s in enumerate(range(first, first + count)):
        st = lib.qed_step(g.ctx, parts, flds[j], dt, seed, s)
        if st != qed.QED_OK:
            raise qed.QedError(st, "qed_step")


def cpu_baseline(workloads, budget_s):
    """The oracle driving the same workload on the host's cores: the full initial
    population (float inputs as the GPU holds them), step after step with appends
    and photon removal, until the time budget is used (at least one step)."""
    import oracle
    threads = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
    w = workloads.c2()
    sp = {}
    for name in ("electrons", "positrons", "photons"):
        s = {k: v.copy() for k, v in w[name].items()}
        for k in ("ux", "uy", "uz", "w"):
            s[k] = s[k].astype(np.float32).astype(np.float64)
        sp[name] = s
    keys = ("x", "y", "z", "ux", "uy", "uz", "w", "id")

    def append(dst, ch, sel):
        for k, ck in zip(keys, ("x", "y", "z", "px", "py", "pz", "w", "id")):
            dst[k] = np.concatenate([dst[k], ch[ck][sel]])

    sub = 0
    steps = 0
    t0 = time.perf_counter()
    while steps == 0 or time.perf_counter() - t0 < budget_s:
        fld = {k: np.float32(v).astype(np.float64) for k, v in workloads.c2_field(steps).items()}
        ch_g, alive, _, _, tg = oracle.photon_step(sp["photons"], fld, w["dt"], w["seed"], steps,
                                                   rng_bits=24, threads=threads)
        ch_e, _, _, te = oracle.lepton_step(sp["electrons"], fld, -1.0, w["dt"], w["seed"], steps,
                                            rng_bits=24, threads=threads)
        ch_p, _, _, tp = oracle.lepton_step(sp["positrons"], fld, 1.0, w["dt"], w["seed"], steps,
                                            rng_bits=24, threads=threads)
        keep = alive.astype(bool)
        sp["photons"] = {k: v[keep] for k, v in sp["photons"].items()}
        append(sp["electrons"], ch_g, ch_g["kind"] == 1)
        append(sp["positrons"], ch_g, ch_g["kind"] == 2)
        append(sp["photons"], ch_e, slice(None))
        append(sp["photons"], ch_p, slice(None))
        sub += tg["substeps"] + te["substeps"] + tp["substeps"]
        steps += 1
    dt = time.perf_counter() - t0
    return {"value": sub / dt, "unit": "particle-sub-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the same workload (1,048,576 e- + 262,144 photons, growing) for its first {steps} "
                      f"steps, FP64 oracle with the same random streams, {dt:.1f} s wall"}


def roofline(kt, st, K):
    """Roofline of the kernel with the largest share of the profiled time."""
    cand = {k: v for k, v in kt.items() if k in ("k_lepton", "k_light", "k_heavy", "k_photon")}
    name = max(cand, key=lambda k: cand[k][1])
    nl, tms = cand[name]
    avg_s = tms * 1e-3 / max(nl, 1)
    lep_sub = st.substeps[0] + st.substeps[1]
    lep_part = st.particles[0] + st.particles[1]
    if name == "k_lepton":
        sub, part, em = lep_sub, lep_part, st.emissions
        byts = BYTES_PER_LEPTON_STEP * part + BYTES_PER_EMISSION * em
        flops = FLOPS_PER_LEPTON_SUBSTEP * sub
    elif name == "k_heavy":
        sub, part = st.heavy_substeps, st.heavy_particles
        em = st.emissions * sub / max(lep_sub, 1)      # emissions shared in proportion to sub-steps
        byts = (BYTES_PER_LEPTON_STEP + BYTES_PER_BINNED_EXTRA) * part + BYTES_PER_EMISSION * em
        flops = FLOPS_PER_LEPTON_SUBSTEP * sub
    elif name == "k_light":
        sub, part = lep_sub - st.heavy_substeps, lep_part - st.heavy_particles
        em = st.emissions * sub / max(lep_sub, 1)
        byts = BYTES_PER_LEPTON_STEP * part + 4 * lep_part + BYTES_PER_EMISSION * em
        flops = FLOPS_PER_LEPTON_SUBSTEP * sub
    else:
        sub, part, em = st.substeps[2], st.particles[2], st.pairs
        byts = BYTES_PER_PHOTON_STEP * part + 2 * BYTES_PER_EMISSION * em
        flops = FLOPS_PER_PHOTON_SUBSTEP * sub
    byts /= max(nl, 1)
    flops /= max(nl, 1)
    t_mem = byts / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (FP32_VECTOR_PEAK_TFLOPS * 1e12)
    if t_mem >= t_alu:
        roof = {"bound": "hbm", "achieved": byts / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = name
    roof["avg_launch_us"] = avg_s * 1e6
    roof["per_launch"] = {"particles": part / max(nl, 1), "substeps": sub / max(nl, 1),
                          "events": em / max(nl, 1), "algorithmic_bytes": byts, "algorithmic_flops": flops}
    return roof


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--scheduler", choices=("naive", "binned"), default="naive")
    ap.add_argument("--no-graph", action="store_true", help="launch steps eagerly in the timed pass")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_2008_10468_amd import qed

    torch.cuda.set_device(0)
    K, W = args.steps, args.warmup
    sched = qed.QED_SCHED_BINNED if args.scheduler == "binned" else qed.QED_SCHED_NAIVE
    stream = torch.cuda.Stream()
    w, g, field = c2_setup(torch, qed, workloads, max(K, W), sched, stream)
    log(f"bench: C2 workload, {w['electrons']['id'].size} e- + {w['photons']['id'].size} photons, "
        f"dt={w['dt']}, steps={K}, warmup={W}")

    # warm-up on the workload (this also sizes the library's scratch), then restore
    # the initial state
    g.load_state(w)
    torch.cuda.synchronize()
    run_steps(qed, g, field, w, 0, W)
    st, rep = g.sync()
    assert st == qed.QED_OK, qed.status_string(st)
    graph = None
    if not args.no_graph:
        # all K steps recorded once into one HIP graph; the timed pass replays it
        assert qed.qed_graph_begin(g.ctx) == qed.QED_OK
        run_steps(qed, g, field, w, 0, K)
        st, graph = qed.qed_graph_end(g.ctx)
        assert st == qed.QED_OK, qed.status_string(st)

    def timed(profile):
        g.load_state(w)
        qed.qed_reset_stats(g.ctx)
        qed.qed_profile_enable(g.ctx, profile)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if graph is not None and not profile:
            assert qed.qed_graph_launch(g.ctx, graph) == qed.QED_OK
        else:
            run_steps(qed, g, field, w, 0, K)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st, rep = g.sync()
        assert st == qed.QED_OK, (qed.status_string(st), list(rep.required_capacity))
        stats = g.stats()
        kt = qed.qed_profile_read(g.ctx) if profile else {}
        qed.qed_profile_enable(g.ctx, 0)
        return ms, stats, rep, kt

    ms, stats, rep, _ = timed(False)
    ms_p, stats_p, _, kt = timed(True)
    sub = sum(stats.substeps)
    ev = stats.emissions + stats.pairs
    value = sub / (ms * 1e-3)
    log(f"bench: {ms:.3f} ms for {K} steps; sub-steps e-/e+/g = {list(stats.substeps)}; "
        f"particle-steps {list(stats.particles)}; emissions {stats.emissions}, pairs {stats.pairs}; "
        f"final counts {list(rep.n)}")
    log("bench: kernel times (profiled pass): " +
        ", ".join(f"{k}: {v[1] / max(v[0], 1) * 1e3:.1f} us x{v[0]}" for k, v in kt.items()))

    roof = roofline(kt, stats_p, K)
    out = {
        "metric": "particle-sub-steps/s",
        "value": value,
        "unit": "particle-sub-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "C2: 1,048,576 e- + 262,144 photons, uniform E = 1e-3 E_S rotating with period "
                        "200 steps, emission + pair creation, mixed precision (f32 push and synchrotron "
                        "functions, f64 sub-step count and positions), buffers growing by appends",
            "steps": K, "p_max": 0.01, "dt_hbar_over_mc2": w["dt"], "seed": w["seed"],
            "scheduler": args.scheduler,
            "launch": "eager" if graph is None else "one HIP graph of all timed steps",
        },
        "events_per_s": ev / (ms * 1e-3),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(workloads, args.cpu_seconds)
    if graph is not None:
        qed.qed_graph_destroy(graph)
    g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
