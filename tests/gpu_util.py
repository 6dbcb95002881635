"""Helpers for the GPU parity tests: run one step on the GPU through the C ABI,
run the oracle on exactly the inputs the GPU saw, and compare particle by particle."""
import numpy as np

import oracle
from paper_2008_10468_amd import qed

RNG_BITS = {qed.QED_PREC_F64: 53, qed.QED_PREC_MIXED: 24}


def as_precision(fields, precision):
    """Field values as the GPU stores them (float32 for the mixed path), in float64."""
    out = {}
    for k, v in fields.items():
        v = np.asarray(v, np.float64)
        out[k] = v.astype(np.float32).astype(np.float64) if precision == qed.QED_PREC_MIXED else v
    return out


def gpu_step(g, fields_host, dt, seed, step):
    """One GPU step.  Returns (before, after, events, status)."""
    before = [g.sp[s].download() for s in range(3)]
    n0 = [b["id"].size for b in before]
    g.step(dt, seed, step)
    st, rep = g.sync()
    after = [g.sp[s].download() for s in range(3)]
    events = [g.sp[s].events_host(n0[s]) if g.sp[s].events is not None else None for s in range(3)]
    return before, after, events, st, rep


def oracle_step(before, fields_host, dt, seed, step, precision, emission=True, pairs=True, p_max=0.01,
                pair_coef=0.1, threads=None):
    """The oracle from the GPU's start-of-step state (float values exact in float64)."""
    rb = RNG_BITS[precision]
    res = {}
    strip = lambda d: {k: d[k].copy() for k in ("x", "y", "z", "ux", "uy", "uz", "w", "id")}
    st_e, st_p, st_g = strip(before[0]), strip(before[1]), strip(before[2])
    fe = fields_host[0]
    fp = fields_host[1]
    fg = fields_host[2]
    if pairs:
        ch, alive, nsub, nev, tl = oracle.photon_step(st_g, fg, dt, seed, step, p_max=p_max, rng_bits=rb,
                                                      pair_coef=pair_coef, threads=threads)
        res["photon"] = (st_g, ch, alive, nsub, nev, tl)
    if emission:
        res["electron"] = (st_e,) + oracle.lepton_step(st_e, fe, -1.0, dt, seed, step, p_max=p_max,
                                                        rng_bits=rb, threads=threads)
        res["positron"] = (st_p,) + oracle.lepton_step(st_p, fp, +1.0, dt, seed, step, p_max=p_max,
                                                        rng_bits=rb, threads=threads)
    return res


def rel(a, b, floor):
    return np.abs(a - b) / np.maximum(np.maximum(np.abs(a), np.abs(b)), floor)


def compare_leptons(after_gpu, events_gpu, orc_state, orc_nev, n0, rtol, min_agree):
    """Per-slot comparison of pre-existing leptons.  Returns the agreement fraction.
    rtol: scalar or per-particle array (float rounding in the push grows with the
    number of sub-steps)."""
    same = events_gpu[:n0] == orc_nev[:n0]
    agree = float(np.mean(same)) if n0 else 1.0
    assert agree >= min_agree, (agree, np.flatnonzero(~same)[:10])
    if n0:
        u_g = np.stack([after_gpu[k][:n0] for k in ("ux", "uy", "uz")])
        u_o = np.stack([orc_state[k][:n0] for k in ("ux", "uy", "uz")])
        umag = np.maximum(np.linalg.norm(u_o, axis=0), 1.0)
        du = np.linalg.norm(u_g - u_o, axis=0) / umag
        tol = np.broadcast_to(np.asarray(rtol, np.float64), du.shape)
        bad = same & (du > tol)
        assert not bad.any(), (du[bad][:5], tol[bad][:5])
    return agree


def compare_children(gpu_ids, gpu_mom, gpu_w, orc_ids, orc_mom, orc_w, rtol, max_missing):
    """Children matched by id (deterministic keys).  Momenta compared on the common set."""
    gi = {int(v): j for j, v in enumerate(gpu_ids)}
    oi = {int(v): j for j, v in enumerate(orc_ids)}
    common = sorted(set(gi) & set(oi))
    missing = len(set(gi) ^ set(oi))
    assert missing <= max_missing, (missing, len(gi), len(oi))
    if common:
        a = np.array([gi[k] for k in common])
        b = np.array([oi[k] for k in common])
        pg = gpu_mom[:, a]
        po = orc_mom[:, b]
        mag = np.maximum(np.linalg.norm(po, axis=0), 1e-30)
        d = np.linalg.norm(pg - po, axis=0) / mag
        assert np.max(d) <= rtol, np.max(d)
        assert np.array_equal(gpu_w[a], orc_w[b])
    return len(common), missing
