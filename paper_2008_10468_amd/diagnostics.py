"""Diagnostics of the generator on synthetic workloads.

* ``event_gaps``: Fig. 1 of Sec. 3.1.1, the histogram of events by the number of
  sub-steps since the particle's previous event (the bound of Sec. 3.1.1 is meant to
  keep few events far from the previous one: 1.5% at 10 or more sub-steps in the
  paper's runs with the refined estimates).
* ``pmax_sensitivity``: the same steps at several P_max (Sec. 3.1.1 ties the sub-step
  count to P_max; the event statistics should not depend on it, the cost should scale
  like 1/P_max).
* ``precision_comparison``: FP64 against mixed precision on one population (Sec. 1 and
  3.2: synchrotron functions to about 1e-8, single-precision accuracy, give simulation
  results almost identical to the 1e-14 ones).
* ``cell_comparison``: sub-steps chosen per particle against sub-steps chosen per cell
  (Algorithms 1 and 2 compute the sub-step for the current cell; the generator's
  default is each particle's own), at several cell sizes: the event statistics should
  not change, the cell's count is the largest of its particles', so the cost grows
  with the particles per cell.

Each returns a dict; ``python -m paper_2008_10468_amd.diagnostics --what fig1`` (or
``pmax``, ``precision``, ``cells``) prints it as one JSON line.  These run the library only; the
tests compare them with the oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import qed


def _torch():
    import torch
    return torch


def _photon_stats(g, initial_ids):
    """Energies of the photons emitted during the run (those whose id is not among the
    initial photons'; compaction moves photons between slots, so slots do not tell)."""
    ph = g.sp[2].download()
    new = ~np.isin(ph["id"], initial_ids)
    k = np.sqrt(ph["ux"][new] ** 2 + ph["uy"][new] ** 2 + ph["uz"][new] ** 2)
    return float(k.mean()) if k.size else 0.0, k


def _capacity(n, steps):
    """Buffer sizes for `steps` steps of a population of n = (e-, e+, photons): room for
    four emissions per lepton and step, and for pairs from one photon in eight a step."""
    pairs = (n[0] + n[1] + n[2]) * steps // 8
    return (max(16, 2 * n[0] + pairs + 1024), max(16, 2 * n[1] + pairs + 1024),
            max(16, 4 * (n[0] + n[1] + n[2]) * steps + 1024))


def event_gaps(state, fields, dt, steps, seed=1, precision=qed.QED_PREC_MIXED, nbins=32, pairs=True,
               capacity=None):
    """Run `steps` steps of `state` with the event-gap histogram on; returns the
    emission and pair histograms and the share of events 10 or more sub-steps after
    the previous one."""
    torch = _torch()
    n = [state[s]["id"].size for s in qed.SPECIES]
    cap = capacity or _capacity(n, steps)
    g = qed.Generator(precision=precision, capacity=cap, pairs=pairs, parent=False, events=False)
    g.load_state(state)
    g.set_fields(fields)
    hist = torch.zeros(2 * nbins, dtype=torch.int64, device="cuda")
    assert qed.qed_event_gaps(g.ctx, hist.data_ptr(), nbins) == qed.QED_OK
    for s in range(steps):
        g.step(dt, seed, s)
    st, rep = g.sync()
    if st != qed.QED_OK:
        raise qed.QedError(st, "qed_sync")
    h = hist.cpu().numpy().reshape(2, nbins)
    stats = g.stats()
    g.close()
    out = {"nbins": nbins, "emission_gaps": h[0].tolist(), "pair_gaps": h[1].tolist(),
           "emissions": int(stats.emissions), "pairs": int(stats.pairs)}
    for name, hh in (("emission", h[0]), ("pair", h[1])):
        tot = int(hh.sum())
        out[f"{name}_share_gap_ge_10"] = float(hh[10:].sum() / tot) if tot else None
    return out


def pmax_sensitivity(state, fields, dt, steps, p_values=(0.003, 0.01, 0.03, 0.1), seed=1,
                     precision=qed.QED_PREC_MIXED, pairs=True):
    """The same steps at several P_max: events, sub-steps, mean photon energy and time."""
    torch = _torch()
    n = [state[s]["id"].size for s in qed.SPECIES]
    cap = _capacity(n, steps + 1)
    rows = []
    for p in p_values:
        stream = torch.cuda.Stream()
        g = qed.Generator(precision=precision, capacity=cap, pairs=pairs, p_max=p, parent=False, events=False,
                          stream=stream.cuda_stream)
        g.load_state(state)
        g.set_fields(fields)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            g.step(dt, seed, s)
        st, rep = g.sync()
        ms = (time.perf_counter() - t0) * 1e3
        if st != qed.QED_OK:
            raise qed.QedError(st, "qed_sync")
        stats = g.stats()
        mean_k, k = _photon_stats(g, state["photons"]["id"])
        rows.append({"p_max": p, "emissions": int(stats.emissions), "pairs": int(stats.pairs),
                     "photon_energy_sem": float(k.std() / np.sqrt(k.size)) if k.size else 0.0,
                     "lepton_substeps": int(stats.substeps[0] + stats.substeps[1]),
                     "photon_substeps": int(stats.substeps[2]), "clips": int(stats.clips),
                     "mean_photon_energy": mean_k, "ms": ms})
        g.close()
    return {"steps": steps, "rows": rows}


def precision_comparison(state, fields, dt, steps, seed=1, pairs=True):
    """FP64 and mixed precision from the same state: event counts and the emitted
    photons' energies (the two use different random streams, 53- and 24-bit draws, so
    they agree in distribution, not photon by photon)."""
    n = [state[s]["id"].size for s in qed.SPECIES]
    cap = _capacity(n, steps + 1)
    out = {}
    for name, prec in (("f64", qed.QED_PREC_F64), ("mixed", qed.QED_PREC_MIXED)):
        g = qed.Generator(precision=prec, capacity=cap, pairs=pairs, parent=False, events=False)
        g.load_state(state)
        g.set_fields(fields)
        for s in range(steps):
            g.step(dt, seed, s)
        st, rep = g.sync()
        if st != qed.QED_OK:
            raise qed.QedError(st, "qed_sync")
        stats = g.stats()
        mean_k, k = _photon_stats(g, state["photons"]["id"])
        out[name] = {"emissions": int(stats.emissions), "pairs": int(stats.pairs), "mean_photon_energy": mean_k,
                     "photon_energy_quantiles": np.quantile(k, [0.1, 0.5, 0.9]).tolist() if k.size else [],
                     "photon_energies": k}
        g.close()
    return out


def cell_comparison(state, fields, dt, steps, cells=(None, 32, 16, 8, 4), seed=1, precision=qed.QED_PREC_MIXED,
                    pairs=True, pos_scale=1.0e4):
    """The same steps with per-particle sub-steps (None) and with sub-steps per cell for
    n^3 cells over the cube [-pos_scale, pos_scale)^3 (n in cells): events, sub-steps,
    mean photon energy and time."""
    torch = _torch()
    n = [state[s]["id"].size for s in qed.SPECIES]
    cap = _capacity(n, steps + 1)
    rows = []
    for nc in cells:
        stream = torch.cuda.Stream()
        g = qed.Generator(precision=precision, capacity=cap, pairs=pairs, parent=False, events=False,
                          stream=stream.cuda_stream)
        g.load_state(state)
        g.set_fields(fields)
        if nc is not None:
            d = 2.0 * pos_scale / nc
            geom = {"nx": nc, "ny": nc, "nz": nc, "x0": -pos_scale, "y0": -pos_scale, "z0": -pos_scale,
                    "dx": d, "dy": d, "dz": d}
            st = qed.qed_substep_cells(g.ctx, geom)
            if st != qed.QED_OK:
                raise qed.QedError(st, "qed_substep_cells")
        # one untimed step (first launches, scratch), then the run from the same state
        g.step(dt, seed, 0)
        g.sync()
        g.load_state(state)
        qed.qed_reset_stats(g.ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            g.step(dt, seed, s)
        st, rep = g.sync()
        ms = (time.perf_counter() - t0) * 1e3
        if st != qed.QED_OK:
            raise qed.QedError(st, "qed_sync")
        stats = g.stats()
        mean_k, k = _photon_stats(g, state["photons"]["id"])
        rows.append({"cells_per_axis": nc, "leptons_per_cell": None if nc is None else (n[0] + n[1]) / nc ** 3,
                     "emissions": int(stats.emissions), "pairs": int(stats.pairs),
                     "lepton_substeps": int(stats.substeps[0] + stats.substeps[1]),
                     "photon_substeps": int(stats.substeps[2]), "mean_photon_energy": mean_k,
                     "photon_energy_sem": float(k.std() / np.sqrt(k.size)) if k.size else 0.0, "ms": ms})
        g.close()
    return {"steps": steps, "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser(description="Diagnostics of the QED generator on synthetic workloads")
    ap.add_argument("--what", choices=("fig1", "pmax", "precision", "cells"), default="fig1")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--n", type=int, default=1 << 16, help="electrons (photons: a quarter)")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads
    torch = _torch()
    torch.cuda.set_device(0)
    w = workloads.c2(n_e=args.n, n_g=args.n // 4)
    state = {s: w[s] for s in qed.SPECIES}
    if args.what == "fig1":
        res = {"c2": event_gaps(state, w["fields"], w["dt"], args.steps)}
        c1 = workloads.c1(n=min(args.n, 16384))
        res["c1_f64"] = event_gaps({s: c1[s] for s in qed.SPECIES}, c1["fields"], c1["dt"], args.steps,
                                   precision=qed.QED_PREC_F64, pairs=False)
    elif args.what == "pmax":
        res = pmax_sensitivity(state, w["fields"], w["dt"], args.steps)
    elif args.what == "cells":
        res = cell_comparison(state, w["fields"], w["dt"], args.steps)
    else:
        res = precision_comparison(state, w["fields"], w["dt"], args.steps)
        from scipy import stats as sps
        res["ks_pvalue_photon_energy"] = float(sps.ks_2samp(res["f64"]["photon_energies"],
                                                            res["mixed"]["photon_energies"]).pvalue)
        for v in ("f64", "mixed"):
            del res[v]["photon_energies"]
    res["workload"] = f"C2 population scaled to {args.n} electrons, {args.steps} steps, field of step 0"
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
