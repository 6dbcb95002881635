#!/usr/bin/env python3
"""Throughput of the QED event generator on one MI355X.

Default workload (``--workload hotspot``): the uneven batch of 16,777,216 electrons
(90% in a weak field with one sub-step each, 10% in a Gaussian hot spot of chi up to
about 100 with up to 1000 sub-steps), per-particle static magnetic fields, emission
only, mixed precision.  A step is one global step of Algorithm 1 over every
electron, run four ways on the same population: the plain generator with the naive
and the binned (persistent, chi-binned) schedulers, and the optical-depth path
(surrogate) with the binned scheduler, its photon energies by rejection and by the
learned inverse CDF (the network shipped for gfx950).  ``value`` is the surrogate's
throughput in the plain generator's unit of work: the particle-sub-steps Algorithm 1
takes for this population (P_max = 0.01, counted on the device in the plain binned
run) per second of surrogate step time; events/s and every run's own figures sit
beside it.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  --gpus above 1 is refused: the path runs on one GPU.
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
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector peak (packed FP32)
FP64_VECTOR_PEAK_TFLOPS = 78.6

# Algorithmic work per unit, counted from the kernel source (mixed precision).
# Floating-point operations: FMA = 2, each reciprocal / square root / cube root /
# logarithm / exponential = 1.  Lepton sub-steps by field kind (the kernels run a
# specialised push and chi for a pure E and a pure B field):
#   Boris push: general 52, pure E 6, pure B 46; gamma and move 15;
#   chi: general 40, pure E 16, pure B 15;
#   plain (Algorithm 1): candidate 14, F and G 37, acceptance 12;
#   optical depth: rate fit 17, rate times 1/gamma 1, optical-depth update 2.
FLOPS_PUSH = {"general": 52, "pure_e": 6, "pure_b": 46}
FLOPS_CHI = {"general": 40, "pure_e": 16, "pure_b": 15}
FLOPS_MOVE = 15
FLOPS_PLAIN_TEST = 14 + 37 + 12
FLOPS_SURR_RATE = 17 + 1 + 2
FLOPS_MLP_PER_EVENT = 2 * (2 * 64 + 64 * 64 + 64 * 64 + 64)   # matrix cores (bf16), reported apart
# per emission on the optical-depth path (vector unit): gamma, chi and the rate fit at the
# crossing and again after the recoil (2 x 44), the next optical depth's logarithm (25,
# double), x from the sample and the photon and recoil (35), the held rotation (20)
FLOPS_SURR_EVENT = 2 * 44 + 25 + 35 + 20
# per learned emission: the network's float layers (layer 1: 64 x (2 fma + activation 4);
# the hidden activations: 64 x (bias + 4); output: 64 x (bias + 4 + fma 2) + 2)
FLOPS_MLP_VALU_PER_EVENT = 64 * 8 + 64 * 5 + 64 * 7 + 2
FLOPS_PER_PHOTON_SUBSTEP = 62       # move 6, candidate 6, F and G 37, acceptance 13
# optical-depth path in a pure magnetic field: the sub-steps up to each crossing (and up to
# the end of the step) are taken in closed form, one advance each: float 57 (axis, the
# parallel and normal parts, the turned momentum and the summed move) and double about 145
# (|t|, the turn's complex step, binary powering over about six bits of m at 20 each, the
# geometric sum, the crossing sub-step tau / d)
FLOPS_SURR_ADVANCE_PURE_B = 57 + 145
BYTES_PER_LEPTON_STEP = 80          # read u 12 + id 8 + position 24; write u 12 + position 24
BYTES_FIELD_PER_PARTICLE = 24       # six float field values, per-particle (stride 1) fields only
BYTES_TAU = 16                      # optical depth read and written (double)
BYTES_PER_EMISSION = 52             # weight read 4; position 24 + k 12 + weight 4 + id 8 written
BYTES_PER_PHOTON_READ = 36          # k 12 + position 24
BYTES_PER_PHOTON_WRITE = 25         # position 24 + flag 1
FLOPS_PER_PHOTON_MOVE = 6           # three fused multiply-adds per sub-step
BYTES_PER_BINNED_EXTRA = 8          # sub-step count read 4 + queue entry read 4 (heavy pass)
BYTES_PER_PAIR = 104                # two lepton records (position 24, u 12, weight 4, id 8) + dead-list entry 8


def flops_per_lepton_substep(field_kind, surrogate=False):
    base = FLOPS_PUSH[field_kind] + FLOPS_MOVE + FLOPS_CHI[field_kind]
    return base + (FLOPS_SURR_RATE if surrogate else FLOPS_PLAIN_TEST)


SCHEDULERS = {"naive": lambda q: q.QED_SCHED_NAIVE, "binned": lambda q: q.QED_SCHED_BINNED,
              "tiled": lambda q: q.QED_SCHED_TILED}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def c2_setup(torch, qed, workloads, steps_total, sched, stream=None, surrogate=False):
    w = workloads.c2()
    sur = qed.QED_SAMPLER_SURROGATE if surrogate else qed.QED_SAMPLER_REJECTION
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 23, 1 << 23, 1 << 25),
                      parent=False, events=False, scheduler=sched,
                      stream=None if stream is None else stream.cuda_stream, sampler=sur, pair_sampler=sur)
    if surrogate:
        m = np.load(os.path.join(ROOT, "paper_2008_10468_amd", "models", "sampler_gfx950.npz"))
        st = qed.qed_sampler_set(g.ctx, m["params"], m["fallback"], float(m["log10_chi_lo"]),
                                 float(m["log10_chi_hi"]))
        assert st == qed.QED_OK, st
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


def kernel_source_hash():
    """SHA-256 over the sources of the generator's kernels (qed_kernels.hip and the
    headers and tables it includes), in name order: identifies the kernels a counter
    summary was taken from."""
    import hashlib
    d = os.path.join(ROOT, "paper_2008_10468_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f == "qed_kernels.hip" or f.endswith((".hpp", ".inc")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, workload, run="-", steps=None):
    """Calibrated HBM bytes per launch of `kernel` in `run` of this workload from the
    committed counter summary, or None if there is none, it was taken over another
    number of steps, or the kernels changed since it was taken.  The summary's lines
    read `source_sha256: <hash>`, `steps: <K>` and `traffic <run> <kernel> <bytes>`."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    sha, val, k = None, None, None
    for line in open(path):
        if line.startswith("source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("steps:"):
            k = int(line.split(":", 1)[1])
        parts = line.split()
        if len(parts) == 4 and parts[0] == "traffic" and parts[1] == run and parts[2] == kernel:
            val = float(parts[3])
    if sha != kernel_source_hash() or (steps is not None and k != steps):
        return None
    return val


def roofline(kt, st, K, workload, field_kind="general", surrogate=False, field_bytes=0, peaks=None,
             kernel=None, run="-"):
    """Roofline of the kernel with the largest share of the profiled time (or `kernel`):
    its algorithmic bytes and flops per launch from the device counters and the unit
    costs above, against 8 TB/s or the FP32 vector peak (and the measured peaks, if
    given); `traffic` from that workload's committed counter summary, if there is one."""
    cand = {k: v for k, v in kt.items()
            if k in ("k_lepton", "k_tiled", "k_light", "k_heavy", "k_photon")}
    name = kernel if kernel in cand else max(cand, key=lambda k: cand[k][1])
    nl, tms = cand[name]
    avg_s = tms * 1e-3 / max(nl, 1)
    lep_sub = st.substeps[0] + st.substeps[1]
    lep_part = st.particles[0] + st.particles[1]
    f_sub = flops_per_lepton_substep(field_kind, surrogate)
    rec = BYTES_PER_LEPTON_STEP + field_bytes + (BYTES_TAU if surrogate else 0)
    mfma = 0.0
    if name in ("k_lepton", "k_tiled"):
        sub, part, em = lep_sub, lep_part, st.emissions
        byts = rec * part + BYTES_PER_EMISSION * em
        flops = f_sub * sub
        learned = st.learned_events
    elif name == "k_heavy":
        sub, part = st.heavy_substeps, st.heavy_particles
        share = sub / max(lep_sub, 1)
        em = st.emissions * share                      # emissions shared in proportion to sub-steps
        learned = st.learned_events * share
        byts = (rec + BYTES_PER_BINNED_EXTRA) * part + BYTES_PER_EMISSION * em
        flops = f_sub * sub
        if surrogate and field_kind == "pure_b":
            # one closed-form advance per crossing and one to the end of the step
            flops = FLOPS_SURR_ADVANCE_PURE_B * (part + em)
    elif name == "k_light":
        sub, part = lep_sub - st.heavy_substeps, lep_part - st.heavy_particles
        share = sub / max(lep_sub, 1)
        em = st.emissions * share
        learned = st.learned_events * share
        byts = rec * part + 4 * lep_part + BYTES_PER_EMISSION * em
        flops = f_sub * sub
    else:  # k_photon: every photon is read and written back (position, flag); the ones
        # that can decay also run the sampling loop (from their record kept in LDS);
        # each pair writes two lepton records and a dead-list entry
        part, sub, em = st.particles[2], st.substeps[2], st.pairs
        learned = 0
        byts = (BYTES_PER_PHOTON_READ + BYTES_PER_PHOTON_WRITE) * part + BYTES_PER_PAIR * em
        flops = FLOPS_PER_PHOTON_MOVE * (sub - st.sampled_substeps) + FLOPS_PER_PHOTON_SUBSTEP * st.sampled_substeps
    if surrogate:
        mfma = FLOPS_MLP_PER_EVENT * learned
        # the emissions' own work: every event, the network's float layers for the learned
        # ones, a candidate test per rejection draw for the others
        if name != "k_photon":
            draws = st.fallback_draws * (em / max(st.emissions, 1))
            flops += FLOPS_SURR_EVENT * em + FLOPS_MLP_VALU_PER_EVENT * learned + FLOPS_PLAIN_TEST * draws
    byts /= max(nl, 1)
    flops /= max(nl, 1)
    mfma /= max(nl, 1)
    t_mem = byts / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (FP32_VECTOR_PEAK_TFLOPS * 1e12)
    if t_mem >= t_alu:
        roof = {"bound": "hbm", "achieved": byts / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        meas = peaks.get("hbm_copy_GBps") if peaks else None
    else:
        roof = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
        meas = peaks.get("fp32_fma_TFLOPs") if peaks else None
    roof["frac"] = roof["achieved"] / roof["peak"]
    if meas:
        roof["measured_peak"] = meas
        roof["frac_of_measured_peak"] = roof["achieved"] / meas
    roof["traffic"] = measured_traffic(name, workload, run, K)
    roof["kernel"] = name
    roof["avg_launch_us"] = avg_s * 1e6
    roof["per_launch"] = {"particles": part / max(nl, 1), "substeps": sub / max(nl, 1),
                          "events": em / max(nl, 1), "algorithmic_bytes": byts, "algorithmic_flops": flops,
                          "flops_per_substep": f_sub}
    if surrogate:
        roof["per_launch"]["mfma_flops"] = mfma
        roof["mfma_tflops"] = mfma / avg_s / 1e12
    return roof


def load_tuning(qed, g, key, path):
    """Apply the autotuner's choice for this workload and scheduler, if recorded (key: one
    "<workload>/<scheduler>" or a list of them, the first recorded one applies)."""
    if not path or not os.path.exists(path):
        return None
    table = json.load(open(path))
    keys = [key] if isinstance(key, str) else list(key)
    choice = next((table[k] for k in keys if table.get(k)), None)
    if not choice:
        return None
    t = qed.qed_get_tuning(g.ctx)
    for k, v in choice["tuning"].items():
        setattr(t, k, int(v))
    assert qed.qed_set_tuning(g.ctx, t) == qed.QED_OK, choice
    return choice["tuning"]


def stepped(torch, qed, g, stream, fields_for_step, state, dt, seed, K, W, use_graph):
    """Warm-up, graph capture, a timed pass and a profiled pass of K steps from state."""
    import ctypes as C
    lib = qed.load()

    def run(first, count):
        parts = C.byref(g.particles())
        flds = [fields_for_step(s) for s in range(first, first + count)]
        for j, s in enumerate(range(first, first + count)):
            st = lib.qed_step(g.ctx, parts, flds[j], float(dt), int(seed), s)
            if st != qed.QED_OK:
                raise qed.QedError(st, "qed_step")

    g.load_state(state)
    torch.cuda.synchronize()
    run(0, W)
    st, rep = g.sync()
    assert st == qed.QED_OK, (qed.status_string(st), list(rep.required_capacity))
    graph = None
    if use_graph:
        assert qed.qed_graph_begin(g.ctx) == qed.QED_OK
        run(0, K)
        st, graph = qed.qed_graph_end(g.ctx)
        assert st == qed.QED_OK, qed.status_string(st)

    def timed(profile):
        g.load_state(state)
        qed.qed_reset_stats(g.ctx)
        qed.qed_profile_enable(g.ctx, profile)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if graph is not None and not profile:
            assert qed.qed_graph_launch(g.ctx, graph) == qed.QED_OK
        else:
            run(0, K)
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
    _, stats_p, _, kt = timed(True)
    if graph is not None:
        qed.qed_graph_destroy(graph)
    log(f"bench: {ms:.3f} ms for {K} steps; sub-steps e-/e+/g = {list(stats.substeps)}; "
        f"particle-steps {list(stats.particles)}; sampled photons {stats.sampled_photons}; "
        f"emissions {stats.emissions}, pairs {stats.pairs}; "
        f"final counts {list(rep.n)}")
    log("bench: kernel times (profiled pass): " +
        ", ".join(f"{k}: {v[1] / max(v[0], 1) * 1e3:.1f} us x{v[0]}" for k, v in kt.items()))
    return ms, stats, stats_p, kt, graph is not None


def header(args, value, ms, K, W, dtype, config, metric="particle-sub-steps/s"):
    return {"metric": metric, "value": value, "unit": metric, "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": config}


def host_cpu():
    """The host's CPU model and core counts (for the oracle baseline's record)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cores": affinity,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def measure_peaks(torch, stream):
    """Measured peaks of this GPU (libqed_peaks.so): HBM copy bandwidth over 2 x 4 GiB,
    and the issue rates of non-packed FP32 and of FP64 fused multiply-adds."""
    import ctypes as C
    path = os.path.join(ROOT, "paper_2008_10468_amd", "libqed_peaks.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2008_10468_amd.build`")
    L = C.CDLL(path)
    L.qed_peak_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int, C.c_void_p, C.POINTER(C.c_float)]
    L.qed_peak_fma.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_uint64, C.c_void_p, C.POINTER(C.c_float),
                               C.POINTER(C.c_double)]
    nbytes = 4 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    ms = C.c_float()
    assert L.qed_peak_copy(a.data_ptr(), b.data_ptr(), nbytes, 10, C.c_void_p(stream.cuda_stream), C.byref(ms)) == 0
    del a, b
    torch.cuda.empty_cache()
    out = {"hbm_copy_GBps": 2 * nbytes / (ms.value * 1e-3) / 1e9}
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    for dtype, key, iters in ((0, "fp32_fma_TFLOPs", 4000), (1, "fp64_fma_TFLOPs", 4000)):
        blocks = ncu * 16
        sink = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
        fl = C.c_double()
        assert L.qed_peak_fma(dtype, sink.data_ptr(), blocks, iters, C.c_void_p(stream.cuda_stream),
                              C.byref(ms), C.byref(fl)) == 0
        out[key] = fl.value / (ms.value * 1e-3) / 1e12
        del sink
    out["spec"] = {"hbm_GBps": HBM_PEAK_GBS, "fp32_vector_TFLOPs": FP32_VECTOR_PEAK_TFLOPS,
                   "fp32_vector_non_packed_TFLOPs": FP32_VECTOR_PEAK_TFLOPS / 2,
                   "fp64_vector_TFLOPs": FP64_VECTOR_PEAK_TFLOPS}
    log(f"bench: measured peaks {out}")
    return out


def cpu_baseline_hotspot(workloads, budget_s, n_sample=1 << 16):
    """The oracle (plain Algorithm 1, FP64, 24-bit uniforms as the mixed path draws
    them) on a stratified sample of the hot-spot population: 2^16 electrons, hot and
    cold in the population's proportions (10% / 90%), with their own per-particle
    fields and float momenta, step after step until the budget is used (at most the
    workload's 50 steps); particle-sub-steps per second of wall time on the threads
    the oracle runs (every core this process may use, within OMP_NUM_THREADS)."""
    import oracle
    w = workloads.c3()
    rng = np.random.default_rng(12345)
    hot = np.flatnonzero(w["hot"])
    cold = np.flatnonzero(~w["hot"])
    n_hot = int(round(n_sample * hot.size / (hot.size + cold.size)))
    sel = np.sort(np.concatenate([rng.choice(hot, n_hot, replace=False),
                                  rng.choice(cold, n_sample - n_hot, replace=False)]))
    st = workloads.subset(w["electrons"], sel)
    for k in ("ux", "uy", "uz", "w"):
        st[k] = st[k].astype(np.float32).astype(np.float64)
    fl = {k: v.astype(np.float32).astype(np.float64)
          for k, v in workloads.field_subset(w["fields"], sel).items()}
    del w
    threads = oracle.default_threads()
    sub = ev = steps = 0
    t0 = time.perf_counter()
    while steps < 50 and (steps == 0 or time.perf_counter() - t0 < budget_s):
        _, _, _, tl = oracle.lepton_step(st, fl, -1.0, workloads.DT_C3, 1, steps, rng_bits=24, threads=threads)
        sub += tl["substeps"]
        ev += tl["events"]
        steps += 1
    dt = time.perf_counter() - t0
    out = {"value": sub / dt, "unit": "particle-sub-steps/s", "cores": threads, "kind": "oracle",
           "sample": f"stratified 2^16-electron sample of the hot-spot population ({n_hot} hot, "
                     f"{n_sample - n_hot} cold), plain Algorithm 1 in FP64 with the same random streams, "
                     f"{steps} steps, {dt:.1f} s wall, {sub} particle-sub-steps",
           "events_per_s": ev / dt}
    out.update(host_cpu())
    return out


def hotspot_tuning_keys(surrogate, net, sched, weak=False):
    """Tuning table keys of a hot-spot run: c3 (plain generator), c5 (optical-depth path
    with the network), c5r (optical-depth path with rejection energies; each sampler at
    the launch shapes and resolve batch tuned for it, c5's if c5r is not recorded); for
    the weak uniform field w5 and w5r first."""
    if not surrogate:
        return [f"c3/{sched}"]
    keys = [f"c5/{sched}"] if net else [f"c5r/{sched}", f"c5/{sched}"]
    if weak:
        keys = ([f"w5/{sched}"] if net else [f"w5r/{sched}", f"w5/{sched}"]) + keys
    return keys


def bench_hotspot(args, torch, qed, workloads):
    """The hot-spot workload (16.8M electrons, 10% hot), four runs on the same population:
    plain naive, plain binned, surrogate binned with rejection energies, surrogate binned
    with the shipped network (the `value`)."""
    K, W = (args.steps if args.steps_given else 20), args.warmup
    n = int(args.c3_particles)
    stream = torch.cuda.Stream()
    peaks = measure_peaks(torch, stream)
    m = np.load(os.path.join(ROOT, "paper_2008_10468_amd", "models", "sampler_gfx950.npz"))
    w = workloads.c3(n=n)
    zero = workloads.uniform_field()
    cap_ph = int(min(0.65 * n * max(K, W) + (1 << 23), 1 << 31))   # about 0.55 photons per e- per step
    p_s = args.surrogate_p_max
    rej, sur = qed.QED_SAMPLER_REJECTION, qed.QED_SAMPLER_SURROGATE
    runs, rooflines = {}, {}
    # name, scheduler, sampler, network installed
    plan = (("plain_naive", qed.QED_SCHED_NAIVE, rej, False), ("plain_binned", qed.QED_SCHED_BINNED, rej, False),
            ("surrogate_rejection_binned", qed.QED_SCHED_BINNED, sur, False),
            ("surrogate_binned", qed.QED_SCHED_BINNED, sur, True))
    for name, sched, sampler, net in plan:
        if args.skip_naive and name == "plain_naive":
            continue
        g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, 16, cap_ph), pairs=False, parent=False,
                          events=False, scheduler=sched, stream=stream.cuda_stream, sampler=sampler,
                          surrogate_p_max=p_s)
        if net:
            assert qed.qed_sampler_set(g.ctx, m["params"], m["fallback"], float(m["log10_chi_lo"]),
                                       float(m["log10_chi_hi"])) == qed.QED_OK
        sname = "naive" if sched == qed.QED_SCHED_NAIVE else "binned"
        tuned = load_tuning(qed, g, hotspot_tuning_keys(sampler == sur, net, sname), args.tuning)
        g.set_fields(None, per_species=[w["fields"], zero, zero])
        fl = [f.struct() for f in g.fields]
        fields = lambda s: (qed.qed_field * 3)(*fl)
        log(f"bench: hot spot, {name}, {n} e-, steps={K}, warmup={W}, tuning={tuned}")
        ms, stats, stats_p, kt, graphed = stepped(torch, qed, g, stream, fields, w, w["dt"], w["seed"], K, W,
                                                  not args.no_graph)
        surr = sampler == sur
        runs[name] = {"ms_per_step": ms / K, "substeps_per_step": sum(stats.substeps) / K,
                      "substeps_per_s": sum(stats.substeps) / (ms * 1e-3),
                      "events_per_s": stats.emissions / (ms * 1e-3), "emissions_per_step": stats.emissions / K,
                      "lepton_substep_target": p_s if surr else 0.01, "tuning": tuned,
                      "learned_events": stats.learned_events, "fallback_events": stats.fallback_events,
                      "fallback_draws": stats.fallback_draws,
                      "kernel_us": {k: v[1] * 1e3 / max(v[0], 1) for k, v in kt.items()},
                      "launch": "one HIP graph of all timed steps" if graphed else "eager"}
        rooflines[name] = roofline(kt, stats_p, K, "hotspot", field_kind="pure_b", surrogate=surr,
                                   field_bytes=BYTES_FIELD_PER_PARTICLE, peaks=peaks, kernel="k_heavy", run=name)
        g.close()
        del g
        torch.cuda.empty_cache()
    best = runs["surrogate_binned"]
    plain_sub = runs["plain_binned"]["substeps_per_step"]
    value = plain_sub / (best["ms_per_step"] * 1e-3)
    out = header(args, value, best["ms_per_step"] * K, K, W, "f32+bf16", {
        "workload": f"hot spot: {n} electrons, gamma log-uniform [1e3, 1e4], isotropic; 90% in B = 5e-7 E_S, "
                    f"10% in a Gaussian hot spot B = 1e-2 exp(-r^2/2) E_S (chi up to ~100, up to 1000 "
                    f"sub-steps), per-particle static fields, emission only, mixed precision; optical-depth "
                    f"path with the learned sampler (sub-step target {p_s}), binned scheduler",
        "value_counts": "the particle-sub-steps Algorithm 1 takes for this population at P_max = 0.01 "
                        "(device count of the plain binned run) per second of the surrogate's step time",
        "steps": K, "dt_hbar_over_mc2": w["dt"], "seed": w["seed"], "scheduler": "binned",
        "tuning": best["tuning"], "launch": best["launch"]})
    out["events_per_s"] = best["events_per_s"]
    out["runs"] = runs
    speed = lambda a, b: runs[b]["ms_per_step"] / runs[a]["ms_per_step"]
    if "plain_naive" in runs:
        out["step_speedup_vs_plain_naive"] = speed("surrogate_binned", "plain_naive")
    out["step_speedup_vs_plain_binned"] = speed("surrogate_binned", "plain_binned")
    out["network_gain_vs_rejection"] = speed("surrogate_binned", "surrogate_rejection_binned")
    out["roofline"] = rooflines["surrogate_binned"]
    out["roofline_plain_binned"] = rooflines["plain_binned"]
    out["peaks"] = peaks
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_hotspot(workloads, args.cpu_seconds)
    return out


def bench_c2(args, torch, qed, workloads):
    K, W = args.steps, args.warmup
    sched = SCHEDULERS[args.scheduler](qed)
    stream = torch.cuda.Stream()
    w, g, field = c2_setup(torch, qed, workloads, max(K, W), sched, stream)
    tuned = load_tuning(qed, g, f"c2/{args.scheduler}", args.tuning)
    log(f"bench: C2 workload, {w['electrons']['id'].size} e- + {w['photons']['id'].size} photons, "
        f"dt={w['dt']}, steps={K}, warmup={W}, tuning={tuned}")
    fields = lambda s: (qed.qed_field * 3)(field(s), field(s), field(s))
    ms, stats, stats_p, kt, graphed = stepped(torch, qed, g, stream, fields, w, w["dt"], w["seed"], K, W,
                                              not args.no_graph)
    sub = sum(stats.substeps)
    out = header(args, sub / (ms * 1e-3), ms, K, W, "f32", {
        "workload": "C2: 1,048,576 e- + 262,144 photons, uniform E = 1e-3 E_S rotating with period "
                    "200 steps, emission + pair creation, mixed precision (f32 push and synchrotron "
                    "functions, f64 sub-step count and positions), buffers growing by appends",
        "steps": K, "p_max": 0.01, "dt_hbar_over_mc2": w["dt"], "seed": w["seed"],
        "scheduler": args.scheduler, "tuning": tuned,
        "launch": "one HIP graph of all timed steps" if graphed else "eager"})
    out["events_per_s"] = (stats.emissions + stats.pairs) / (ms * 1e-3)
    out["roofline"] = roofline(kt, stats_p, K, "c2", field_kind="pure_e")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(workloads, args.cpu_seconds)
    g.close()
    return out


def bench_weak(args, torch, qed, workloads):
    """The learned sampler where rejection is expensive: 16.8M electrons in one weak
    uniform field (chi 1e-3 to 1e-2), the optical-depth path with the shipped network
    against the same path with rejection energies, the plain generator (binned) beside."""
    K, W = (args.steps if args.steps_given else 20), args.warmup
    n = int(args.c3_particles)
    m = np.load(os.path.join(ROOT, "paper_2008_10468_amd", "models", "sampler_gfx950.npz"))
    w = workloads.weak(n=n)
    zero = workloads.uniform_field()
    cap_ph = int(min(1.0 * n * max(K, W) + (1 << 23), 1 << 31))
    p_s = args.surrogate_p_max
    rej, sur = qed.QED_SAMPLER_REJECTION, qed.QED_SAMPLER_SURROGATE
    stream = torch.cuda.Stream()
    runs = {}
    for name, sampler, net in (("plain_binned", rej, False), ("surrogate_rejection_binned", sur, False),
                               ("surrogate_binned", sur, True)):
        g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, 16, cap_ph), pairs=False, parent=False,
                          events=False, scheduler=qed.QED_SCHED_BINNED, stream=stream.cuda_stream, sampler=sampler,
                          surrogate_p_max=p_s)
        if net:
            assert qed.qed_sampler_set(g.ctx, m["params"], m["fallback"], float(m["log10_chi_lo"]),
                                       float(m["log10_chi_hi"])) == qed.QED_OK
        tuned = load_tuning(qed, g, hotspot_tuning_keys(sampler == sur, net, "binned", weak=True), args.tuning)
        g.set_fields(None, per_species=[w["fields"], zero, zero])
        fl = [f.struct() for f in g.fields]
        fields = lambda s: (qed.qed_field * 3)(*fl)
        log(f"bench: weak field, {name}, {n} e-, steps={K}, warmup={W}, tuning={tuned}")
        ms, stats, stats_p, kt, graphed = stepped(torch, qed, g, stream, fields, w, w["dt"], w["seed"], K, W,
                                                  not args.no_graph)
        runs[name] = {"ms_per_step": ms / K, "substeps_per_step": sum(stats.substeps) / K,
                      "emissions_per_step": stats.emissions / K, "events_per_s": stats.emissions / (ms * 1e-3),
                      "learned_events": stats.learned_events, "fallback_events": stats.fallback_events,
                      "fallback_draws": stats.fallback_draws, "tuning": tuned,
                      "kernel_us": {k: v[1] * 1e3 / max(v[0], 1) for k, v in kt.items()}}
        g.close()
        del g
        torch.cuda.empty_cache()
    best = runs["surrogate_binned"]
    value = runs["plain_binned"]["substeps_per_step"] / (best["ms_per_step"] * 1e-3)
    out = header(args, value, best["ms_per_step"] * K, K, W, "f32+bf16", {
        "workload": f"weak field: {n} electrons, gamma log-uniform [1e3, 1e4], isotropic, uniform B = 1e-6 E_S "
                    f"(chi 1e-3 to 1e-2), emission only, mixed precision; optical-depth path with the learned "
                    f"sampler (sub-step target {p_s}), binned scheduler",
        "value_counts": "the particle-sub-steps Algorithm 1 takes for this population at P_max = 0.01 per "
                        "second of the optical-depth path's step time",
        "steps": K, "dt_hbar_over_mc2": w["dt"], "seed": w["seed"], "scheduler": "binned"})
    out["runs"] = runs
    speed = lambda a, b: runs[b]["ms_per_step"] / runs[a]["ms_per_step"]
    out["network_gain_vs_rejection"] = speed("surrogate_binned", "surrogate_rejection_binned")
    out["step_speedup_vs_plain_binned"] = speed("surrogate_binned", "plain_binned")
    rj = runs["surrogate_rejection_binned"]
    out["rejection_draws_per_energy"] = rj["fallback_draws"] / max(rj["fallback_events"], 1)
    return out


def bench_c2s(args, torch, qed, workloads):
    """C2 on the optical-depth paths (leptons: optical depth, network shipped for gfx950,
    sub-step target 0.1; photons: exact decay time, no sub-steps) against the plain
    generator on the same population and fields."""
    K, W = args.steps, args.warmup
    runs = {}
    for name, surrogate in (("plain_naive", False), ("surrogate_naive", True)):
        stream = torch.cuda.Stream()
        w, g, field = c2_setup(torch, qed, workloads, max(K, W), qed.QED_SCHED_NAIVE, stream, surrogate)
        tuned = load_tuning(qed, g, "c2s/naive" if surrogate else "c2/naive", args.tuning)
        log(f"bench: C2 {name}")
        fields = lambda s: (qed.qed_field * 3)(field(s), field(s), field(s))
        ms, stats, stats_p, kt, graphed = stepped(torch, qed, g, stream, fields, w, w["dt"], w["seed"], K, W,
                                                  not args.no_graph)
        runs[name] = {"ms_per_step": ms / K, "substeps_per_step": sum(stats.substeps) / K,
                      "substeps_per_s": sum(stats.substeps) / (ms * 1e-3),
                      "events_per_s": (stats.emissions + stats.pairs) / (ms * 1e-3),
                      "emissions": stats.emissions, "pairs": stats.pairs, "tuning": tuned,
                      "kernel_us": {k: v[1] * 1e3 / max(v[0], 1) for k, v in kt.items()}}
        g.close()
        del g
        torch.cuda.empty_cache()
    best = runs["surrogate_naive"]
    out = header(args, best["substeps_per_s"], best["ms_per_step"] * K, K, W, "f32+bf16", {
        "workload": "C2 on the optical-depth paths: 1,048,576 e- + 262,144 photons, uniform E = 1e-3 E_S "
                    "rotating with period 200 steps; leptons by optical depth with the learned sampler "
                    "(sub-step target 0.1), photons by exact decay time; plain generator beside it",
        "steps": K, "dt_hbar_over_mc2": workloads.DT_C2, "seed": 1})
    out["runs"] = runs
    out["step_speedup_vs_plain"] = runs["plain_naive"]["ms_per_step"] / best["ms_per_step"]
    out["events_per_s"] = best["events_per_s"]
    return out


def bench_c1(args, torch, qed, workloads):
    """FP64 correctness configuration: 16,384 electrons in a uniform static B field."""
    K, W = (args.steps if args.steps_given else 100), args.warmup
    w = workloads.c1()
    stream = torch.cuda.Stream()
    sched = SCHEDULERS[args.scheduler](qed)
    g = qed.Generator(precision=qed.QED_PREC_F64, capacity=(16384, 16, 1 << 22), pairs=False,
                      parent=False, events=False, scheduler=sched, stream=stream.cuda_stream)
    g.set_fields(w["fields"])
    f = g.fields[0].struct()
    fields = lambda s: (qed.qed_field * 3)(f, f, f)
    ms, stats, stats_p, kt, graphed = stepped(torch, qed, g, stream, fields, w, w["dt"], w["seed"], K, W,
                                              not args.no_graph)
    out = header(args, sum(stats.substeps) / (ms * 1e-3), ms, K, W, "f64", {
        "workload": "C1: 16,384 electrons, gamma log-uniform [1e2, 1e4], isotropic, uniform B = 1e-3 E_S, "
                    "emission only, FP64", "steps": K, "dt_hbar_over_mc2": w["dt"],
        "scheduler": args.scheduler})
    out["events_per_s"] = stats.emissions / (ms * 1e-3)
    g.close()
    return out


def bench_c3(args, torch, qed, workloads):
    """Uneven batch: 16,777,216 electrons, 10% in a Gaussian hot spot (chi up to 100)."""
    K, W = (args.steps if args.steps_given else 50), args.warmup
    n = int(args.c3_particles)
    w = workloads.c3(n=n)
    stream = torch.cuda.Stream()
    sched = SCHEDULERS[args.scheduler](qed)
    cap_ph = int(min(0.65 * n * max(K, W) + (1 << 23), 1 << 31))   # about 0.55 photons per e- per step
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, 16, cap_ph), pairs=False, parent=False,
                      events=False, scheduler=sched, stream=stream.cuda_stream)
    tuned = load_tuning(qed, g, f"c3/{args.scheduler}", args.tuning)
    zero = workloads.uniform_field()
    g.set_fields(None, per_species=[w["fields"], zero, zero])
    fl = [f.struct() for f in g.fields]
    fields = lambda s: (qed.qed_field * 3)(*fl)
    log(f"bench: C3 workload, {n} e-, hot fraction 0.1, dt={w['dt']}, steps={K}, tuning={tuned}")
    ms, stats, stats_p, kt, graphed = stepped(torch, qed, g, stream, fields, w, w["dt"], w["seed"], K, W,
                                              not args.no_graph)
    out = header(args, sum(stats.substeps) / (ms * 1e-3), ms, K, W, "f32", {
        "workload": f"C3: {n} electrons, 90% in B = 5e-7 E_S, 10% in a Gaussian hot spot "
                    "B = 1e-2 exp(-r^2/2) E_S (chi up to ~100), per-particle static fields, emission only, "
                    "mixed precision", "steps": K, "dt_hbar_over_mc2": w["dt"],
        "scheduler": args.scheduler, "tuning": tuned,
        "launch": "one HIP graph of all timed steps" if graphed else "eager"})
    out["events_per_s"] = stats.emissions / (ms * 1e-3)
    out["roofline"] = roofline(kt, stats_p, K, "c3", field_kind="pure_b", field_bytes=BYTES_FIELD_PER_PARTICLE)
    g.close()
    return out


def bench_c4(args, torch, qed, workloads):
    """Synchrotron-function microbenchmark: F and G of 2^28 log-uniform x in [1e-4, 50]."""
    n = 1 << int(args.c4_log2n)
    cfg = qed.qed_config_default()
    stream = torch.cuda.Stream()
    cfg.stream = stream.cuda_stream
    ctx = qed.qed_init(cfg)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    res = {}
    for dtype in (torch.float32, torch.float64):
        u = torch.rand(n, generator=gen, device="cuda", dtype=torch.float64)
        x = (10.0 ** (-4.0 + u * (math.log10(50.0) + 4.0))).to(dtype)
        del u
        F = torch.empty_like(x)
        G = torch.empty_like(x)
        qd = qed.QED_F32 if dtype == torch.float32 else qed.QED_F64
        for _ in range(2):
            assert qed.qed_synchrotron(ctx, x.data_ptr(), F.data_ptr(), G.data_ptr(), n, qd) == qed.QED_OK
        torch.cuda.synchronize()
        reps = 5
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            qed.qed_synchrotron(ctx, x.data_ptr(), F.data_ptr(), G.data_ptr(), n, qd)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        assert qed.qed_sync(ctx)[0] == qed.QED_OK
        bpe = 3 * x.element_size()
        res[str(dtype).split(".")[-1]] = {"evals_per_s": n / (ms * 1e-3), "ms": ms,
                                          "hbm_GBps": n * bpe / (ms * 1e-3) / 1e9}
        log(f"bench: C4 {dtype}: {ms:.3f} ms for {n} evaluations, {res[str(dtype).split('.')[-1]]}")
        del x, F, G
    qed.qed_finalize(ctx)
    r32 = res["float32"]
    out = header(args, r32["evals_per_s"], r32["ms"], 1, 2, "f32", {
        "workload": f"C4: F and G of 2^{args.c4_log2n} x log-uniform in [1e-4, 50], resident in HBM"},
        metric="evaluations/s")
    out["per_dtype"] = res
    out["roofline"] = {"bound": "hbm", "achieved": r32["hbm_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": r32["hbm_GBps"] / HBM_PEAK_GBS, "traffic": None,
                       "kernel": "k_synchrotron<float>", "avg_launch_us": r32["ms"] * 1e3}
    return out


def bench_c5(args, torch, qed, workloads):
    """Learned sampler: train the network on this GPU, then run the hot-spot workload
    with the surrogate (optical depth + network, binned scheduler) against the plain
    rejection generator (naive and binned)."""
    K, W = (args.steps if args.steps_given else 20), args.warmup
    n = int(args.c3_particles)
    ctx = qed.qed_init(qed.qed_config_default())
    tc = qed.qed_train_config_default()
    t0 = time.perf_counter()
    params, loss, err, fb = qed.qed_train_sampler(ctx, tc)
    train_s = time.perf_counter() - t0
    qed.qed_finalize(ctx)
    batch = tc.blocks * 64 * tc.batch_tiles
    log(f"bench: trained in {train_s:.2f} s ({tc.steps} steps x {batch} samples); final loss {loss[-1]:.3e}; "
        f"bins above {tc.tolerance}: {int(fb.sum())} of {tc.nbins}; max bin error {err.max():.2e}")
    if args.save_model:
        np.savez(args.save_model, params=params, fallback=fb, bin_err=err, loss=loss,
                 log10_chi_lo=tc.log10_chi_lo, log10_chi_hi=tc.log10_chi_hi)
    w = workloads.c3(n=n)
    zero = workloads.uniform_field()
    cap_ph = int(min(0.65 * n * max(K, W) + (1 << 23), 1 << 31))
    runs = {}
    p_s = args.surrogate_p_max
    rej, sur = qed.QED_SAMPLER_REJECTION, qed.QED_SAMPLER_SURROGATE
    # name, scheduler, sampler, surrogate sub-step target, network installed
    for name, sched, sampler, ps, net in (("plain_naive", qed.QED_SCHED_NAIVE, rej, p_s, False),
                                          ("plain_binned", qed.QED_SCHED_BINNED, rej, p_s, False),
                                          ("surrogate_plain_substeps_binned", qed.QED_SCHED_BINNED, sur, 0.01, True),
                                          ("surrogate_rejection_binned", qed.QED_SCHED_BINNED, sur, p_s, False),
                                          ("surrogate_binned", qed.QED_SCHED_BINNED, sur, p_s, True)):
        stream = torch.cuda.Stream()
        g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, 16, cap_ph), pairs=False, parent=False,
                          events=False, scheduler=sched, stream=stream.cuda_stream, sampler=sampler,
                          surrogate_p_max=ps)
        if net:
            assert qed.qed_sampler_set(g.ctx, params, fb, tc.log10_chi_lo, tc.log10_chi_hi) == qed.QED_OK
        sname = "naive" if sched == qed.QED_SCHED_NAIVE else "binned"
        tuned = load_tuning(qed, g, hotspot_tuning_keys(sampler == sur, net, sname), args.tuning)
        g.set_fields(None, per_species=[w["fields"], zero, zero])
        fl = [f.struct() for f in g.fields]
        fields = lambda s: (qed.qed_field * 3)(*fl)
        log(f"bench: C5 {name}")
        ms, stats, stats_p, kt, graphed = stepped(torch, qed, g, stream, fields, w, w["dt"], w["seed"], K, W,
                                                  not args.no_graph)
        runs[name] = {"substeps_per_s": sum(stats.substeps) / (ms * 1e-3), "ms_per_step": ms / K,
                      "substeps_per_step": sum(stats.substeps) / K,
                      "lepton_substep_target": ps if sampler == sur else 0.01, "tuning": tuned,
                      "events_per_s": stats.emissions / (ms * 1e-3), "emissions": stats.emissions,
                      "learned_events": stats.learned_events, "fallback_events": stats.fallback_events,
                      "fallback_draws": stats.fallback_draws}
        g.close()
        del g
        torch.cuda.empty_cache()
    best = runs["surrogate_binned"]
    out = header(args, best["substeps_per_s"], best["ms_per_step"] * K, K, W, "f32+bf16", {
        "workload": f"C5: learned sampler (2-64-64-64-1, bf16 hidden layers) deployed in the hot-spot "
                    f"workload ({n} electrons, 10% hot), surrogate + binned vs plain rejection",
        "steps": K, "train_steps": tc.steps, "train_batch": batch, "surrogate_p_max": p_s})
    out["runs"] = runs
    # the surrogate runs fewer sub-steps for the same emission law, so the comparison is by
    # time per step (equal work: the same particles, the same expected emissions)
    speed = lambda a, b: runs[b]["ms_per_step"] / runs[a]["ms_per_step"]
    out["step_speedup_vs_plain_naive"] = speed("surrogate_binned", "plain_naive")
    out["step_speedup_vs_plain_binned"] = speed("surrogate_binned", "plain_binned")
    out["network_gain_vs_rejection"] = speed("surrogate_binned", "surrogate_rejection_binned")
    out["substep_bound_gain"] = speed("surrogate_binned", "surrogate_plain_substeps_binned")
    out["plain_equivalent_substeps_per_s"] = runs["plain_binned"]["substeps_per_step"] / (best["ms_per_step"] * 1e-3)
    out["training"] = {"seconds": train_s, "samples": tc.steps * batch, "final_loss": float(loss[-1]),
                       "bins": tc.nbins, "fallback_bins": int(fb.sum()), "max_bin_cdf_error": float(err.max()),
                       "median_bin_cdf_error": float(np.median(err))}
    return out


def copy_probe(torch, mib):
    """One plain device copy of known size: its FETCH_SIZE / WRITE_SIZE counter readings
    convert the generator kernels' readings into bytes."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return {"bytes_read": 4 * n, "bytes_written": 4 * n, "ms": ms, "GBps": 8 * n / (ms * 1e-3) / 1e9}


def bench_shower(args, torch, qed, workloads):
    """In-step cascades: 65,536 electrons, positrons and photons each seeding a shower
    (energies 1e4 to 3e5, B = 2e-3 E_S); every step runs the main pass and five
    follow-up passes over the particles created in the previous pass."""
    K, W = (args.steps if args.steps_given else 1), 1    # the population grows several-fold per step
    gens = 5
    n = 1 << 16
    w = workloads.shower(n=n)
    stream = torch.cuda.Stream()
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 22, 1 << 22, 1 << 23), parent=False,
                      events=False, stream=stream.cuda_stream, cascade_generations=gens)
    g.set_fields(w["fields"])
    f = g.fields[0].struct()
    fields = lambda s: (qed.qed_field * 3)(f, f, f)
    log(f"bench: shower workload, {n} of each species, dt={w['dt']}, {gens} cascade passes, steps={K}")
    ms, stats, stats_p, kt, graphed = stepped(torch, qed, g, stream, fields, w, w["dt"], w["seed"], K, W,
                                              not args.no_graph)
    out = header(args, sum(stats.substeps) / (ms * 1e-3), ms, K, W, "f32", {
        "workload": f"shower: {n} electrons, {n} positrons, {n} photons, energies log-uniform [1e4, 3e5], "
                    f"isotropic, uniform B = 2e-3 E_S, {gens} in-step cascade passes, mixed precision",
        "steps": K, "dt_hbar_over_mc2": w["dt"], "cascade_generations": gens,
        "launch": "one HIP graph of all timed steps" if graphed else "eager"})
    out["particle_steps"] = list(stats.particles)
    out["events"] = {"emissions": stats.emissions, "pairs": stats.pairs}
    out["roofline"] = roofline(kt, stats_p, K, "shower", field_kind="pure_b")
    g.close()
    return out


def bench_grid(args, torch, qed, workloads):
    """Grid coupling: gather of the six Yee-grid field components to the particles and
    deposition of their currents, 1,048,576 electrons (the C2 population) in a periodic
    box of 32^3 cells by default (32 particles per cell; --grid-cells 128 gives 0.5), stored in
    cell order as a PIC code keeps them (the figure) and in random order (the worst case)."""
    K = args.steps if args.steps_given else 50
    n, nc = 1 << 20, int(args.grid_cells)
    w = workloads.c2(n_e=n, n_g=16)
    geom = workloads.cell_box(nc)
    e = w["electrons"]
    cell = ((np.floor((e["z"] - geom["z0"]) / geom["dz"]).astype(np.int64) % nc) * nc +
            (np.floor((e["y"] - geom["y0"]) / geom["dy"]).astype(np.int64) % nc)) * nc + \
        (np.floor((e["x"] - geom["x0"]) / geom["dx"]).astype(np.int64) % nc)
    by_cell = workloads.subset(e, np.argsort(cell, kind="stable"))
    stream = torch.cuda.Stream()
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, 16, 16), parent=False, events=False,
                      stream=stream.cuda_stream)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    comps = [torch.randn((nc, nc, nc), generator=gen, device="cuda", dtype=torch.float32) * 1e-3 for _ in range(6)]
    grid = qed.cell_geometry(geom)
    grid.ex, grid.ey, grid.ez, grid.bx, grid.by, grid.bz = [c.data_ptr() for c in comps]
    outs = [torch.empty(n, device="cuda", dtype=torch.float32) for _ in range(6)]
    j = [torch.zeros(nc ** 3, device="cuda", dtype=torch.float64) for _ in range(3)]
    sp = g.sp[0].struct()
    ptrs = [o.data_ptr() for o in outs]

    def timed(fn):
        for _ in range(3):
            assert fn() == qed.QED_OK
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(K):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K

    def sort_min(v):
        t = qed.qed_get_tuning(g.ctx)
        t.deposit_sort_min = v
        assert qed.qed_set_tuning(g.ctx, t) == qed.QED_OK

    times, wave = {}, {}
    default_sort = qed.qed_get_tuning(g.ctx).deposit_sort_min
    for order, pop in (("random", e), ("cell", by_cell)):
        g.load_state({"electrons": pop, "positrons": w["positrons"], "photons": w["photons"]})
        torch.cuda.synchronize()
        dep = lambda: qed.qed_deposit(g.ctx, grid, sp, -1.0, *[t.data_ptr() for t in j])
        times[order] = (timed(lambda: qed.qed_gather(g.ctx, grid, sp, ptrs)), timed(dep))
        sort_min(0xFFFFFFFF)            # the per-wave kernel without the tile sort, for comparison
        wave[order] = timed(dep)
        sort_min(default_sort)
        assert g.sync()[0] == qed.QED_OK
    ms_g, ms_d = times["cell"]
    grid_bytes = 6 * 4 * nc ** 3
    j_bytes = 3 * 8 * nc ** 3
    bytes_g = n * (24 + 6 * 4) + grid_bytes          # positions read, six floats written, the grid once
    bytes_d = n * (24 + 3 * 4 + 4) + 2 * j_bytes     # positions, momenta and weight read, J read and written once
    for order, (tg, td) in times.items():
        log(f"bench: grid {nc}^3, {n} electrons in {order} order: gather {tg * 1e3:.1f} us, "
            f"deposit {td * 1e3:.1f} us per call (per-wave kernel without the sort {wave[order] * 1e3:.1f} us)")
    out = header(args, n / ((ms_g + ms_d) * 1e-3), (ms_g + ms_d) * K, K, 3, "f32+f64", {
        "workload": f"grid coupling: {n} electrons (C2 population, positions uniform over the box, stored in "
                    f"cell order), periodic Yee grid of {nc}^3 cells, float fields, double currents; one gather "
                    f"and one deposit per step", "cells": nc ** 3}, metric="particles/s")
    rd = lambda b, ms: {"bound": "hbm", "achieved": b / (ms * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                        "frac": b / (ms * 1e-3) / 8e12, "traffic": None,
                        "avg_launch_us": ms * 1e3, "algorithmic_bytes": b}
    out["gather"] = rd(bytes_g, ms_g)
    out["deposit"] = rd(bytes_d, ms_d)
    out["random_order_us"] = {"gather": times["random"][0] * 1e3, "deposit": times["random"][1] * 1e3}
    out["deposit_without_tile_sort_us"] = {o: v * 1e3 for o, v in wave.items()}
    dom = "gather" if ms_g >= ms_d else "deposit"
    # the deposit is one call of five kernels (tile sort, LDS sums, reduction); its figure is per call
    out["roofline"] = dict(out[dom], kernel="k_gather" if dom == "gather" else
                           "qed_deposit (k_dep_bin, k_dep_scan, k_dep_scatter, k_dep_accum, k_dep_reduce)")
    g.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=("hotspot", "c2", "c1", "c3", "c4", "c5", "c2s", "shower", "grid", "weak"),
                    default="hotspot")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--scheduler", choices=("naive", "binned", "tiled"), default="naive")
    ap.add_argument("--no-graph", action="store_true", help="launch steps eagerly in the timed pass")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2008_10468_amd", "tuning_gfx950.json"))
    ap.add_argument("--c3-particles", type=float, default=16777216)
    ap.add_argument("--c4-log2n", type=int, default=28)
    ap.add_argument("--grid-cells", type=int, default=32, help="grid: cells per axis of the periodic box")
    ap.add_argument("--save-model", default=None, help="c5: write the trained network to this .npz")
    ap.add_argument("--surrogate-p-max", type=float, default=0.1,
                    help="c5: the surrogate's lepton sub-step target")
    ap.add_argument("--skip-naive", action="store_true", help="hotspot: leave out the plain naive run")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-MiB float buffer once (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the path runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    args.steps_given = args.steps is not None
    if args.steps is None:
        args.steps = 200

    import torch

    import workloads
    from paper_2008_10468_amd import qed

    torch.cuda.set_device(0)
    fn = {"hotspot": bench_hotspot, "c2": bench_c2, "c1": bench_c1, "c3": bench_c3, "c4": bench_c4, "c5": bench_c5,
          "weak": bench_weak,
          "c2s": bench_c2s, "shower": bench_shower, "grid": bench_grid}[args.workload]
    out = fn(args, torch, qed, workloads)
    if args.copy_probe:
        out["copy_probe"] = copy_probe(torch, args.copy_probe)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
