"""FP64 CPU oracle for the QED event generator (arXiv:2008.10468).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this module; the GPU library never
does.  It wraps ``qed_oracle.c`` (plain C, FP64) through ctypes and adds a
thread-pool driver that runs independent particle chunks in parallel (ctypes
releases the GIL during the foreign call).  It shares no code with the GPU path.

Functions follow the paper:
  * ``synchrotron(x)``           F(x)=x int_x^inf K_{5/3}, G(x)=x K_{2/3} (Sec. 3.2.1)
  * ``pm(x, chi, gamma, dt)``    3 x^2 P(x^3) of eq. (1), the acceptance bound of Alg. 1
  * ``pp(x, chi_g, eps_g, dt)``  P_p(x) of eq. (2), bracket order corrected
  * ``bound_emission``/``bound_pair``/``nsub``   sub-step rule of Sec. 3.1.1
  * ``lepton_step``/``photon_step``              Algorithms 1 and 2 over arrays
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qed_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ALPHA = 7.2973525693e-3


def build(force: bool = True) -> str:
    """Compile qed_oracle.c into liboracle.so with gcc (FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("p_max", C.c_double), ("pair_coef", C.c_double),
                ("seed", C.c_uint64), ("step", C.c_uint32), ("n_cap", C.c_uint32),
                ("rng_bits", C.c_int32), ("pad", C.c_int32)]


class Children(C.Structure):
    _fields_ = [("cap", C.c_int64), ("n", C.c_int64)] + \
        [(f, C.POINTER(C.c_double)) for f in ("x", "y", "z", "px", "py", "pz", "w")] + \
        [("id", C.POINTER(C.c_uint64)), ("parent", C.POINTER(C.c_uint64)),
         ("sub", C.POINTER(C.c_uint32)), ("kind", C.POINTER(C.c_int32)), ("tb", C.POINTER(C.c_double))]


class Tally(C.Structure):
    _fields_ = [("substeps", C.c_uint64), ("events", C.c_uint64), ("clips", C.c_uint64),
                ("max_p", C.c_double)]


_lib = None
_lock = threading.Lock()

_D = C.POINTER(C.c_double)
_U64 = C.POINTER(C.c_uint64)
_U32 = C.POINTER(C.c_uint32)
_U8 = C.POINTER(C.c_uint8)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = C.CDLL(_LIB)
            L.orc_philox4x32_10.argtypes = [_U32, _U32, _U32]
            L.orc_philox_vec.argtypes = [C.c_int64, _U32, _U32, _U32]
            L.orc_u53.argtypes = [C.c_uint32, C.c_uint32]
            L.orc_u53.restype = C.c_double
            L.orc_u24.argtypes = [C.c_uint32]
            L.orc_u24.restype = C.c_double
            L.orc_draw_xy.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int,
                                      _D, _D]
            L.orc_child_id.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
            L.orc_child_id.restype = C.c_uint64
            L.orc_synchrotron_vec.argtypes = [C.c_int64, _D, _D, _D]
            for name in ("orc_chi_lepton", "orc_chi_photon"):
                getattr(L, name).argtypes = [_D, _D, _D]
                getattr(L, name).restype = C.c_double
            L.orc_bound_emission.argtypes = [C.c_double] * 3
            L.orc_bound_emission.restype = C.c_double
            L.orc_bound_pair.argtypes = [C.c_double] * 4
            L.orc_bound_pair.restype = C.c_double
            L.orc_nsub.argtypes = [C.c_double, C.c_double, C.c_uint32]
            L.orc_nsub.restype = C.c_uint32
            L.orc_pm.argtypes = [C.c_double] * 4
            L.orc_pm.restype = C.c_double
            L.orc_pp.argtypes = [C.c_double] * 4
            L.orc_pp.restype = C.c_double
            L.orc_boris.argtypes = [_D, _D, _D, C.c_double, C.c_double]
            L.orc_emission_prob.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
            L.orc_emission_prob.restype = C.c_double
            L.orc_emission_energy.argtypes = [C.c_double] * 3
            L.orc_emission_energy.restype = C.c_double
            L.orc_emission_cdf.argtypes = [C.c_double] * 2
            L.orc_emission_cdf.restype = C.c_double
            L.orc_pair_cdf.argtypes = [C.c_double] * 2
            L.orc_pair_cdf.restype = C.c_double
            L.orc_pair_prob.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
            L.orc_pair_prob.restype = C.c_double
            fld = C.POINTER(_D)
            L.orc_lepton_batch.argtypes = [C.POINTER(Params), C.c_double, C.c_int64,
                                           _D, _D, _D, _D, _D, _D, _D, _U64, _D, fld, C.c_int64,
                                           _U32, _U32, C.POINTER(Children), C.POINTER(Tally), _U32]
            L.orc_lepton_batch.restype = C.c_int64
            L.orc_photon_batch.argtypes = [C.POINTER(Params), C.c_int64,
                                           _D, _D, _D, _D, _D, _D, _D, _U64, _D, fld, C.c_int64,
                                           _U8, _U32, _U32, C.POINTER(Children), C.POINTER(Tally), _U32]
            L.orc_photon_batch.restype = C.c_int64
            _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# ---------------------------------------------------------------- scalars

def philox(ctr, key):
    """Philox4x32-10 of counters ctr[...,4] under keys key[...,2] (uint32)."""
    ctr = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    key = np.ascontiguousarray(np.broadcast_to(np.asarray(key, dtype=np.uint32).reshape(-1, 2),
                                               (ctr.shape[0], 2)))
    out = np.empty_like(ctr)
    lib().orc_philox_vec(ctr.shape[0], _p(ctr, C.c_uint32), _p(key, C.c_uint32), _p(out, C.c_uint32))
    return out


def u53(hi, lo):
    return lib().orc_u53(int(hi), int(lo))


def u24(w):
    return lib().orc_u24(int(w))


def draw_xy(seed, pid, step, i, rng_bits):
    x = C.c_double()
    y = C.c_double()
    lib().orc_draw_xy(seed, pid, step, i, rng_bits, C.byref(x), C.byref(y))
    return x.value, y.value


def child_id(seed, parent, step, i, slot):
    return lib().orc_child_id(seed, parent, step, i, slot)


def synchrotron(x):
    """(F, G) = (x int_x^inf K_{5/3}, x K_{2/3}) elementwise, FP64."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    F = np.empty_like(x)
    G = np.empty_like(x)
    lib().orc_synchrotron_vec(x.size, _p(x, C.c_double), _p(F, C.c_double), _p(G, C.c_double))
    return F, G


def synchrotron_parallel(x, threads=None):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    F = np.empty_like(x)
    G = np.empty_like(x)
    threads = threads or default_threads()
    chunks = np.array_split(np.arange(x.size), threads * 4)

    def run(ix):
        if ix.size == 0:
            return
        a, b = int(ix[0]), int(ix[-1]) + 1
        xs = x[a:b]
        lib().orc_synchrotron_vec(b - a, _p(xs, C.c_double),
                                  C.cast(F.ctypes.data + 8 * a, _D), C.cast(G.ctypes.data + 8 * a, _D))

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, chunks))
    return F, G


def chi_lepton(u, E, B):
    a = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (u, E, B)]
    return lib().orc_chi_lepton(*[_p(v, C.c_double) for v in a])


def chi_photon(k, E, B):
    a = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (k, E, B)]
    return lib().orc_chi_photon(*[_p(v, C.c_double) for v in a])


def bound_emission(chi, gamma, dt):
    return lib().orc_bound_emission(chi, gamma, dt)


def bound_pair(chi_g, eps_g, dt, coef=0.1):
    return lib().orc_bound_pair(chi_g, eps_g, dt, coef)


def nsub(f, p_max, n_cap=1 << 24):
    return lib().orc_nsub(f, p_max, n_cap)


def pm(x, chi, gamma, dt):
    return lib().orc_pm(x, chi, gamma, dt)


def pp(x, chi_g, eps_g, dt):
    return lib().orc_pp(x, chi_g, eps_g, dt)


def boris(u, E, B, q, dt):
    u = np.array(u, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    lib().orc_boris(_p(u, C.c_double), _p(E, C.c_double), _p(B, C.c_double), q, dt)
    return u


def emission_prob(chi, gamma, dt, clip=False):
    return lib().orc_emission_prob(chi, gamma, dt, int(clip))


def emission_energy(chi, gamma, dt):
    return lib().orc_emission_energy(chi, gamma, dt)


def emission_cdf(chi, delta):
    return lib().orc_emission_cdf(chi, delta)


def pair_prob(chi_g, eps_g, dt, clip=False):
    return lib().orc_pair_prob(chi_g, eps_g, dt, int(clip))


def pair_cdf(chi_g, x):
    """Normalised CDF of the electron's energy fraction x in pair creation (eq. (2))."""
    return lib().orc_pair_cdf(chi_g, x)


# ---------------------------------------------------------------- batch steps

CHILD_FIELDS = ("x", "y", "z", "px", "py", "pz", "w")


def _children(cap):
    arrs = {f: np.zeros(cap, np.float64) for f in CHILD_FIELDS}
    arrs["id"] = np.zeros(cap, np.uint64)
    arrs["parent"] = np.zeros(cap, np.uint64)
    arrs["sub"] = np.zeros(cap, np.uint32)
    arrs["kind"] = np.zeros(cap, np.int32)
    arrs["tb"] = np.zeros(cap, np.float64)
    c = Children()
    c.cap = cap
    c.n = 0
    for f in CHILD_FIELDS:
        setattr(c, f, _p(arrs[f], C.c_double))
    c.id = _p(arrs["id"], C.c_uint64)
    c.parent = _p(arrs["parent"], C.c_uint64)
    c.sub = _p(arrs["sub"], C.c_uint32)
    c.kind = _p(arrs["kind"], C.c_int32)
    c.tb = _p(arrs["tb"], C.c_double)
    return c, arrs


def _params(dt, p_max, seed, step, rng_bits, pair_coef=0.1, n_cap=1 << 24):
    P = Params()
    P.dt = dt
    P.p_max = p_max
    P.pair_coef = pair_coef
    P.seed = seed
    P.step = step
    P.n_cap = n_cap
    P.rng_bits = rng_bits
    return P


def _fields(fields, n):
    """fields: dict with ex..bz as arrays of length n (per particle) or 1 (uniform)."""
    arrs = [np.ascontiguousarray(np.asarray(fields[k], dtype=np.float64).ravel())
            for k in ("ex", "ey", "ez", "bx", "by", "bz")]
    stride = 0 if arrs[0].size == 1 else 1
    if stride:
        assert all(a.size >= n for a in arrs)
    return arrs, stride


def default_threads():
    """Host threads the oracle uses by default: the cores this process may run on,
    capped by OMP_NUM_THREADS when it is set (a shared host's allotment)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.strip().isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def _run_chunks(n, fn, threads):
    threads = max(1, threads or default_threads())
    nchunk = min(max(1, n // 64), threads * 8) if n else 0
    bounds = np.linspace(0, n, nchunk + 1).astype(np.int64) if nchunk else np.array([0, 0])
    jobs = [(int(bounds[j]), int(bounds[j + 1])) for j in range(len(bounds) - 1)]
    if threads == 1 or len(jobs) <= 1:
        return [fn(a, b) for a, b in jobs]
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda ab: fn(*ab), jobs))


def _merge(results):
    out = {}
    for key in ("x", "y", "z", "px", "py", "pz", "w", "id", "parent", "sub", "kind", "tb"):
        parts = [r[key] for r in results]
        out[key] = np.concatenate(parts) if parts else np.zeros(0)
    return out


def _t0_ptr(t0, a):
    return None if t0 is None else C.cast(t0.ctypes.data + 8 * a, _D)


def _nf_ptr(nf, a):
    return None if nf is None else C.cast(nf.ctypes.data + 4 * a, _U32)


def lepton_step(state, fields, q, dt, seed, step, p_max=0.01, rng_bits=53, n_cap=1 << 24,
                threads=None, t0=None, nsub=None):
    """Algorithm 1 on arrays.  ``state`` has float64 arrays ux,uy,uz,x,y,z,w and uint64 id;
    they are updated in place.  ``t0`` (optional float64 array): each particle's start
    time within the step (it runs over dt - t0).  ``nsub`` (optional uint32 array): the
    number of sub-steps each particle takes instead of its own (0 keeps its own; see
    cell_substeps).  Returns (children dict, per-particle nsub, per-particle event
    counts, tally dict); children carry their birth time tb."""
    if t0 is not None:
        t0 = np.ascontiguousarray(t0, np.float64)
    if nsub is not None:
        nsub = np.ascontiguousarray(nsub, np.uint32)
    n = state["id"].size
    for k in ("ux", "uy", "uz", "x", "y", "z", "w"):
        assert state[k].dtype == np.float64 and state[k].flags.c_contiguous
    fl, stride = _fields(fields, n)
    nsub_a = np.zeros(n, np.uint32)
    nev_a = np.zeros(n, np.uint32)
    P = _params(dt, p_max, seed, step, rng_bits, n_cap=n_cap)

    def run(a, b):
        m = b - a
        fp = (_D * 6)(*[C.cast(f.ctypes.data + 8 * a * stride, _D) for f in fl])
        cap = 64 + 2 * m
        while True:
            ch, arrs = _children(cap)
            tl = Tally()
            saved = {k: state[k][a:b].copy() for k in ("ux", "uy", "uz", "x", "y", "z")}

            def ptr(k, dt_=C.c_double, off=8):
                return C.cast(state[k].ctypes.data + off * a, C.POINTER(dt_))
            bad = lib().orc_lepton_batch(
                C.byref(P), q, m, ptr("ux"), ptr("uy"), ptr("uz"), ptr("x"), ptr("y"), ptr("z"),
                ptr("w"), ptr("id", C.c_uint64), _t0_ptr(t0, a), fp, stride,
                C.cast(nsub_a.ctypes.data + 4 * a, _U32), C.cast(nev_a.ctypes.data + 4 * a, _U32),
                C.byref(ch), C.byref(tl), _nf_ptr(nsub, a))
            if ch.n <= cap:
                break
            for k, v in saved.items():   # rerun the chunk with room for every child
                state[k][a:b] = v
            cap = int(ch.n)
        res = {k: v[:ch.n].copy() for k, v in arrs.items()}
        res["tally"] = (tl.substeps, tl.events, tl.clips, tl.max_p, bad)
        return res

    results = _run_chunks(n, run, threads)
    tally = dict(substeps=sum(r["tally"][0] for r in results),
                 events=sum(r["tally"][1] for r in results),
                 clips=sum(r["tally"][2] for r in results),
                 max_p=max([r["tally"][3] for r in results], default=0.0),
                 nonfinite=sum(r["tally"][4] for r in results))
    return _merge(results), nsub_a, nev_a, tally


def photon_step(state, fields, dt, seed, step, p_max=0.01, rng_bits=53, pair_coef=0.1,
                n_cap=1 << 24, threads=None, t0=None, nsub=None):
    """Algorithm 2 on arrays (state: photon momentum k in ux,uy,uz, and x,y,z,w float64,
    id uint64; updated in place; t0 and nsub as for lepton_step).
    Returns (children dict [kind 1 = e-, 2 = e+], alive mask, nsub, events, tally)."""
    if t0 is not None:
        t0 = np.ascontiguousarray(t0, np.float64)
    if nsub is not None:
        nsub = np.ascontiguousarray(nsub, np.uint32)
    n = state["id"].size
    fl, stride = _fields(fields, n)
    alive = np.ones(n, np.uint8)
    nsub_a = np.zeros(n, np.uint32)
    nev_a = np.zeros(n, np.uint32)
    P = _params(dt, p_max, seed, step, rng_bits, pair_coef=pair_coef, n_cap=n_cap)

    def run(a, b):
        m = b - a
        fp = (_D * 6)(*[C.cast(f.ctypes.data + 8 * a * stride, _D) for f in fl])
        cap = 2 * m + 2
        ch, arrs = _children(cap)
        tl = Tally()

        def ptr(k, dt_=C.c_double, off=8):
            return C.cast(state[k].ctypes.data + off * a, C.POINTER(dt_))
        bad = lib().orc_photon_batch(
            C.byref(P), m, ptr("ux"), ptr("uy"), ptr("uz"), ptr("x"), ptr("y"), ptr("z"),
            ptr("w"), ptr("id", C.c_uint64), _t0_ptr(t0, a), fp, stride,
            C.cast(alive.ctypes.data + a, _U8),
            C.cast(nsub_a.ctypes.data + 4 * a, _U32), C.cast(nev_a.ctypes.data + 4 * a, _U32),
            C.byref(ch), C.byref(tl), _nf_ptr(nsub, a))
        assert ch.n <= cap
        res = {k: v[:ch.n].copy() for k, v in arrs.items()}
        res["tally"] = (tl.substeps, tl.events, tl.clips, tl.max_p, bad)
        return res

    results = _run_chunks(n, run, threads)
    tally = dict(substeps=sum(r["tally"][0] for r in results),
                 events=sum(r["tally"][1] for r in results),
                 clips=sum(r["tally"][2] for r in results),
                 max_p=max([r["tally"][3] for r in results], default=0.0),
                 nonfinite=sum(r["tally"][4] for r in results))
    return _merge(results), alive, nsub_a, nev_a, tally


# ---------------------------------------------------------------- sub-steps per cell

def own_substeps(state, fields, dt, photons=False, p_max=0.01, pair_coef=0.1, n_cap=1 << 24):
    """Step 1 of Algorithm 1 (leptons) or 2 (photons=True) for each particle on its own:
    the sub-step count N = max(1, ceil(f / P_max)) from the bound f of Sec. 3.1.1 over dt,
    one particle at a time; 0 for a particle with non-finite momentum or field."""
    n = state["id"].size
    fl, stride = _fields(fields, n)
    out = np.zeros(n, np.uint32)
    for i in range(n):
        u = np.array([state["ux"][i], state["uy"][i], state["uz"][i]], np.float64)
        E = np.array([fl[0][i * stride], fl[1][i * stride], fl[2][i * stride]])
        B = np.array([fl[3][i * stride], fl[4][i * stride], fl[5][i * stride]])
        if not (np.all(np.isfinite(u)) and np.all(np.isfinite(E)) and np.all(np.isfinite(B))):
            continue
        if photons:
            eps = float(np.sqrt(u @ u))
            out[i] = 1 if eps == 0.0 else nsub(bound_pair(chi_photon(u, E, B), eps, dt, pair_coef), p_max, n_cap)
        else:
            gamma = float(np.sqrt(1.0 + u @ u))
            out[i] = nsub(bound_emission(chi_lepton(u, E, B), gamma, dt), p_max, n_cap)
    return out


def cell_substeps(electrons, positrons, photons, fields, cells, dt, p_max=0.01, pair_coef=0.1,
                  n_cap=1 << 24):
    """Algorithms 1 and 2, step 1, with the sub-step chosen for the current cell: every
    particle's own count (own_substeps, over the whole step dt), then in each cell of
    ``cells`` (a grid geometry, oracle.grid.cell_index) the largest count among its
    electrons and positrons together (Algorithm 1) and, separately, among its photons
    (Algorithm 2).  fields: the three species' fields.  Returns, per species, the count
    each particle takes: its cell's, or its own where its position is not finite or its
    own count is 0 (non-finite input)."""
    from oracle import grid as _grid
    ncell = cells["nx"] * cells["ny"] * cells["nz"]
    sp = (electrons, positrons, photons)
    own = [own_substeps(sp[s], fields[s], dt, photons=(s == 2), p_max=p_max, pair_coef=pair_coef, n_cap=n_cap)
           for s in range(3)]
    cell = [_grid.cell_index(cells, sp[s]["x"], sp[s]["y"], sp[s]["z"]) for s in range(3)]
    best = [np.zeros(ncell, np.uint32), np.zeros(ncell, np.uint32)]   # leptons, photons
    for s in range(3):
        ok = (cell[s] >= 0) & (own[s] > 0)
        np.maximum.at(best[s // 2], cell[s][ok], own[s][ok])
    out = []
    for s in range(3):
        ok = (cell[s] >= 0) & (own[s] > 0)
        n = own[s].copy()
        n[ok] = best[s // 2][cell[s][ok]]
        out.append(n)
    return out


# ---------------------------------------------------------------- cascades

def event_gaps(lepton_children, photon_children, nbins):
    """Fig. 1's diagnostic (Sec. 3.1.1): events counted by the number of sub-steps since
    the particle's previous event in the step (since the step start for its first one).
    lepton_children: children dicts of lepton_step (emissions); photon_children: of
    photon_step (pairs; both children of a decay carry its sub-step).  Gaps >= nbins go
    to the last bin.  Returns (emission histogram, pair histogram), int64 arrays."""
    he = np.zeros(nbins, np.int64)
    hp = np.zeros(nbins, np.int64)
    for ch in lepton_children:
        par = np.asarray(ch["parent"], np.uint64)
        sub = np.asarray(ch["sub"], np.int64)
        order = np.lexsort((sub, par))
        prev_par, prev_sub = None, -1
        for j in order:
            p, k = int(par[j]), int(sub[j])
            gap = k + 1 if p != prev_par else k - prev_sub
            he[min(gap, nbins - 1)] += 1
            prev_par, prev_sub = p, k
    if photon_children is not None:
        sel = np.asarray(photon_children["kind"]) == 1
        for k in np.asarray(photon_children["sub"], np.int64)[sel]:
            hp[min(int(k) + 1, nbins - 1)] += 1
    return he, hp


def _append(dst, ch, sel):
    for k, ck in zip(("x", "y", "z", "ux", "uy", "uz", "w", "id"), ("x", "y", "z", "px", "py", "pz", "w", "id")):
        dst[k] = np.concatenate([dst[k], ch[ck][sel]])


def cascade_step(electrons, positrons, photons, fields, dt, seed, step, generations, p_max=0.01,
                 rng_bits=53, pair_coef=0.1, n_cap=1 << 24, threads=None):
    """One global step with in-step cascades (the generator's follow-up passes): the
    particles present at the step start run over the whole step (Algorithms 2 then 1);
    then, for each of ``generations`` passes, the particles created in the previous
    pass run over the rest of the step, dt - (their birth time), in the same field (a
    dict of uniform values).  Children of the last pass are kept but not moved.
    The species dicts are replaced by the new populations (photons that decayed are
    removed), each with a "birth" array: the time within the step at which the
    particle was created (0 for those present at the start).  Returns (electrons,
    positrons, photons, per-pass tallies)."""
    sp = {"e": {k: v.copy() for k, v in electrons.items()}, "p": {k: v.copy() for k, v in positrons.items()},
          "g": {k: v.copy() for k, v in photons.items()}}
    lo = {k: 0 for k in sp}
    hi = {k: sp[k]["id"].size for k in sp}
    t0 = {k: np.zeros(hi[k]) for k in sp}   # start time of every particle in the step
    alive_all = np.ones(hi["g"], np.uint8)
    tallies = []
    for gen in range(generations + 1):
        sub = {k: {kk: np.ascontiguousarray(v[lo[k]:hi[k]]) for kk, v in sp[k].items()} for k in sp}
        tz = {k: (None if gen == 0 else np.ascontiguousarray(t0[k][lo[k]:hi[k]])) for k in sp}
        chg, alive, _, _, tg = photon_step(sub["g"], fields, dt, seed, step, p_max=p_max, rng_bits=rng_bits,
                                           pair_coef=pair_coef, n_cap=n_cap, threads=threads, t0=tz["g"])
        che, _, _, te = lepton_step(sub["e"], fields, -1.0, dt, seed, step, p_max=p_max, rng_bits=rng_bits,
                                    n_cap=n_cap, threads=threads, t0=tz["e"])
        chp, _, _, tp = lepton_step(sub["p"], fields, 1.0, dt, seed, step, p_max=p_max, rng_bits=rng_bits,
                                    n_cap=n_cap, threads=threads, t0=tz["p"])
        for k in sp:
            for kk in sp[k]:
                sp[k][kk][lo[k]:hi[k]] = sub[k][kk]
        alive_all[lo["g"]:hi["g"]] = alive
        tallies.append((tg, te, tp))
        # children: pairs to the leptons, photons to the photons, with their birth times
        for k, ch, sel in (("e", chg, chg["kind"] == 1), ("p", chg, chg["kind"] == 2)):
            _append(sp[k], ch, sel)
            t0[k] = np.concatenate([t0[k], ch["tb"][sel]])
        for ch in (che, chp):
            _append(sp["g"], ch, slice(None))
            t0["g"] = np.concatenate([t0["g"], ch["tb"]])
        alive_all = np.concatenate([alive_all, np.ones(sp["g"]["id"].size - alive_all.size, np.uint8)])
        for k in sp:
            lo[k], hi[k] = hi[k], sp[k]["id"].size
    for k in sp:
        sp[k]["birth"] = t0[k]
    keep = alive_all.astype(bool)
    sp["g"] = {k: v[keep] for k, v in sp["g"].items()}
    return sp["e"], sp["p"], sp["g"], tallies
