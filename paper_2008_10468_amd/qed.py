"""ctypes binding of libqed.so (include/qed.h).  Argument marshalling only: every
step of the generator runs in the library's HIP kernels; torch provides device
memory and the stream.  Importing this module does not load the library; the
first call does, and fails loudly if it has not been built."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqed.so")

QED_OK, QED_ERR_INVALID_ARG, QED_ERR_CAPACITY, QED_ERR_NONFINITE, QED_ERR_HIP, QED_ERR_STATE = 0, -1, -2, -3, -4, -5
QED_ERR_SCRATCH = -6
QED_STATIC_MAX_SLOTS = 1 << 20
QED_F32, QED_F64 = 0, 1
QED_PREC_F64, QED_PREC_MIXED = 0, 1
QED_SCHED_NAIVE, QED_SCHED_BINNED, QED_SCHED_TILED = 0, 1, 2
QED_SAMPLER_REJECTION, QED_SAMPLER_SURROGATE = 0, 1
QED_MLP_NPARAMS = 8577
QED_MLP_MAX_BINS = 256

SPECIES = ("electrons", "positrons", "photons")


class qed_species(C.Structure):
    _fields_ = [("n", C.c_void_p), ("capacity", C.c_uint64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("ux", C.c_void_p), ("uy", C.c_void_p), ("uz", C.c_void_p),
                ("w", C.c_void_p), ("id", C.c_void_p), ("parent", C.c_void_p),
                ("events", C.c_void_p), ("tau", C.c_void_p), ("birth", C.c_void_p)]


class qed_particles(C.Structure):
    _fields_ = [(s, qed_species) for s in SPECIES]


class qed_field(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ex", "ey", "ez", "bx", "by", "bz")] + [("stride", C.c_uint64)]


class qed_grid(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ex", "ey", "ez", "bx", "by", "bz")] + \
        [("nx", C.c_uint32), ("ny", C.c_uint32), ("nz", C.c_uint32), ("pad", C.c_uint32)] + \
        [(k, C.c_double) for k in ("x0", "y0", "z0", "dx", "dy", "dz")]


class qed_config(C.Structure):
    _fields_ = [("device", C.c_int), ("stream", C.c_void_p), ("precision", C.c_int),
                ("p_max", C.c_double), ("emission", C.c_int), ("pairs", C.c_int),
                ("scheduler", C.c_int), ("pair_bound_coef", C.c_double),
                ("max_substeps", C.c_uint32), ("sampler", C.c_int), ("cascade_generations", C.c_uint32),
                ("surrogate_p_max", C.c_double), ("pair_sampler", C.c_int)]


class qed_report(C.Structure):
    _fields_ = [("status", C.c_int32), ("pad", C.c_int32), ("required_capacity", C.c_uint64 * 3),
                ("nonfinite", C.c_uint64), ("n", C.c_uint64 * 3)]


class qed_stats(C.Structure):
    _fields_ = [("steps", C.c_uint64), ("substeps", C.c_uint64 * 3), ("particles", C.c_uint64 * 3),
                ("heavy_particles", C.c_uint64), ("heavy_substeps", C.c_uint64),
                ("sampled_photons", C.c_uint64), ("sampled_substeps", C.c_uint64), ("emissions", C.c_uint64),
                ("pairs", C.c_uint64), ("clips", C.c_uint64), ("capped", C.c_uint64),
                ("max_p", C.c_double), ("learned_events", C.c_uint64), ("fallback_events", C.c_uint64),
                ("fallback_draws", C.c_uint64), ("envelope_clips", C.c_uint64),
                ("pair_learned", C.c_uint64), ("pair_fallback", C.c_uint64),
                ("pair_fallback_draws", C.c_uint64), ("pair_envelope_clips", C.c_uint64),
                ("chi_guard", C.c_uint64)]


class qed_tuning(C.Structure):
    _fields_ = [("lepton_blocks_per_cu", C.c_uint32), ("heavy_blocks_per_cu", C.c_uint32),
                ("photon_blocks_per_cu", C.c_uint32), ("light_max", C.c_uint32), ("chunk", C.c_uint32),
                ("resolve_batch", C.c_uint32), ("prepass_blocks_per_cu", C.c_uint32),
                ("prepass_finish", C.c_uint32), ("scatter_blocks_per_cu", C.c_uint32),
                ("bins_per_octave", C.c_uint32), ("light_tile", C.c_uint32), ("tiled_slots", C.c_uint32),
                ("deposit_sort_min", C.c_uint32)]


class qed_sampler_model(C.Structure):
    _fields_ = [("params", C.c_void_p), ("fallback", C.c_void_p), ("nbins", C.c_int32), ("pad", C.c_int32),
                ("log10_chi_lo", C.c_double), ("log10_chi_hi", C.c_double)]


class qed_train_config(C.Structure):
    _fields_ = [("log10_chi_lo", C.c_double), ("log10_chi_hi", C.c_double),
                ("table_chi", C.c_uint32), ("table_x", C.c_uint32), ("steps", C.c_uint32),
                ("blocks", C.c_uint32), ("batch_tiles", C.c_uint32), ("lr", C.c_float), ("lr_final", C.c_float),
                ("seed", C.c_uint64), ("nbins", C.c_int32), ("per_bin", C.c_int32), ("tolerance", C.c_double),
                ("target", C.c_int32), ("pad", C.c_int32)]


class qed_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char_p), ("launches", C.c_uint64), ("total_ms", C.c_double)]


EXPORTS = ("qed_config_default", "qed_init", "qed_step", "qed_sync", "qed_synchrotron",
           "qed_get_stats", "qed_reset_stats", "qed_get_tuning", "qed_set_tuning",
           "qed_profile_enable", "qed_profile_read", "qed_graph_begin", "qed_graph_end",
           "qed_graph_launch", "qed_graph_destroy",
           "qed_step_counted", "qed_step_static", "qed_pair_rate", "qed_event_gaps", "qed_substep_cells", "qed_gather", "qed_deposit",
           "qed_pair_sampler_set", "qed_pair_sampler_infer", "qed_sampler_set", "qed_sampler_infer", "qed_emission_rate", "qed_emission_cdf",
           "qed_train_config_default", "qed_train_sampler", "qed_mlp_gradient",
           "qed_finalize", "qed_status_string")

_lib = None


def load(path: str = LIB_PATH):
    """Load libqed.so; raise if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2008_10468_amd.build`")
    L = C.CDLL(path)
    L.qed_config_default.argtypes = [C.POINTER(qed_config)]
    L.qed_init.argtypes = [C.POINTER(C.c_void_p), C.POINTER(qed_config)]
    L.qed_step.argtypes = [C.c_void_p, C.POINTER(qed_particles), C.POINTER(qed_field), C.c_double,
                           C.c_uint64, C.c_uint32]
    L.qed_step_counted.argtypes = [C.c_void_p, C.POINTER(qed_particles), C.POINTER(qed_field), C.c_double,
                                   C.c_uint64, C.c_void_p]
    L.qed_step_static.argtypes = [C.c_void_p, C.POINTER(qed_particles), C.POINTER(qed_field), C.c_double,
                                  C.c_uint64, C.c_uint32]
    L.qed_sync.argtypes = [C.c_void_p, C.POINTER(qed_report)]
    L.qed_synchrotron.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_int]
    L.qed_get_stats.argtypes = [C.c_void_p, C.POINTER(qed_stats)]
    L.qed_reset_stats.argtypes = [C.c_void_p]
    L.qed_get_tuning.argtypes = [C.c_void_p, C.POINTER(qed_tuning)]
    L.qed_set_tuning.argtypes = [C.c_void_p, C.POINTER(qed_tuning)]
    L.qed_profile_enable.argtypes = [C.c_void_p, C.c_int]
    L.qed_profile_read.argtypes = [C.c_void_p, C.POINTER(qed_kernel_time), C.c_int, C.POINTER(C.c_int)]
    L.qed_graph_begin.argtypes = [C.c_void_p]
    L.qed_graph_end.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
    L.qed_graph_launch.argtypes = [C.c_void_p, C.c_void_p]
    L.qed_graph_destroy.argtypes = [C.c_void_p]
    L.qed_graph_destroy.restype = None
    L.qed_sampler_set.argtypes = [C.c_void_p, C.POINTER(qed_sampler_model)]
    L.qed_sampler_infer.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64]
    L.qed_pair_sampler_set.argtypes = [C.c_void_p, C.POINTER(qed_sampler_model)]
    L.qed_pair_sampler_infer.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64]
    L.qed_emission_rate.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64]
    L.qed_pair_rate.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64]
    L.qed_event_gaps.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32]
    L.qed_substep_cells.argtypes = [C.c_void_p, C.POINTER(qed_grid)]
    L.qed_gather.argtypes = [C.c_void_p, C.POINTER(qed_grid), C.POINTER(qed_species), C.c_void_p * 6]
    L.qed_deposit.argtypes = [C.c_void_p, C.POINTER(qed_grid), C.POINTER(qed_species), C.c_double,
                              C.c_void_p, C.c_void_p, C.c_void_p]
    L.qed_emission_cdf.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_uint32, C.c_uint32, C.c_void_p,
                                   C.c_void_p]
    L.qed_train_config_default.argtypes = [C.POINTER(qed_train_config)]
    L.qed_train_sampler.argtypes = [C.c_void_p, C.POINTER(qed_train_config), C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p]
    L.qed_mlp_gradient.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]
    L.qed_finalize.argtypes = [C.c_void_p]
    L.qed_finalize.restype = None
    L.qed_status_string.argtypes = [C.c_int]
    L.qed_status_string.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("qed_finalize", "qed_status_string", "qed_graph_destroy"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class QedError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


def status_string(s):
    return load().qed_status_string(int(s)).decode()


def _check(st, what):
    if st != QED_OK:
        raise QedError(st, what)


# ---------------------------------------------------------------- thin wrappers

def qed_config_default():
    cfg = qed_config()
    _check(load().qed_config_default(C.byref(cfg)), "qed_config_default")
    return cfg


def qed_init(cfg):
    ctx = C.c_void_p()
    _check(load().qed_init(C.byref(ctx), C.byref(cfg)), "qed_init")
    return ctx


def qed_step(ctx, particles, fields, dt, seed, step):
    arr = (qed_field * 3)(*fields)
    return load().qed_step(ctx, C.byref(particles), arr, float(dt), int(seed), int(step))


def qed_step_static(ctx, particles, fields, dt, seed, step):
    arr = (qed_field * 3)(*fields)
    return load().qed_step_static(ctx, C.byref(particles), arr, float(dt), int(seed), int(step))


def qed_step_counted(ctx, particles, fields, dt, seed, step_ptr):
    """step_ptr: device address of a uint32 step counter."""
    arr = (qed_field * 3)(*fields)
    return load().qed_step_counted(ctx, C.byref(particles), arr, float(dt), int(seed), step_ptr)


def qed_sync(ctx):
    rep = qed_report()
    st = load().qed_sync(ctx, C.byref(rep))
    return st, rep


def qed_synchrotron(ctx, x, F, G, n, dtype):
    return load().qed_synchrotron(ctx, x, F, G, int(n), int(dtype))


def qed_get_stats(ctx):
    s = qed_stats()
    _check(load().qed_get_stats(ctx, C.byref(s)), "qed_get_stats")
    return s


def qed_reset_stats(ctx):
    _check(load().qed_reset_stats(ctx), "qed_reset_stats")


def qed_get_tuning(ctx):
    t = qed_tuning()
    _check(load().qed_get_tuning(ctx, C.byref(t)), "qed_get_tuning")
    return t


def qed_set_tuning(ctx, t):
    return load().qed_set_tuning(ctx, C.byref(t))


def qed_profile_enable(ctx, on):
    _check(load().qed_profile_enable(ctx, int(on)), "qed_profile_enable")


def qed_profile_read(ctx):
    """{kernel name: (launches, total ms)} since the last read."""
    arr = (qed_kernel_time * 16)()
    cnt = C.c_int()
    _check(load().qed_profile_read(ctx, arr, 16, C.byref(cnt)), "qed_profile_read")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(cnt.value)}


def qed_graph_begin(ctx):
    return load().qed_graph_begin(ctx)


def qed_graph_end(ctx):
    g = C.c_void_p()
    st = load().qed_graph_end(ctx, C.byref(g))
    return st, g


def qed_graph_launch(ctx, g):
    return load().qed_graph_launch(ctx, g)


def qed_graph_destroy(g):
    load().qed_graph_destroy(g)


def qed_finalize(ctx):
    load().qed_finalize(ctx)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _set_model(fn, ctx, params, fallback, log10_chi_lo, log10_chi_hi):
    if params is None:
        return fn(ctx, None)
    p = np.ascontiguousarray(params, np.float32)
    fb = np.ascontiguousarray(fallback, np.uint8)
    m = qed_sampler_model(params=_ptr(p).value, fallback=_ptr(fb).value, nbins=int(fb.size), pad=0,
                          log10_chi_lo=float(log10_chi_lo), log10_chi_hi=float(log10_chi_hi))
    return fn(ctx, C.byref(m))


def qed_sampler_set(ctx, params=None, fallback=None, log10_chi_lo=-3.0, log10_chi_hi=2.0):
    """Install a model (numpy float32 params, uint8 fallback flags per bin) or remove it (None)."""
    return _set_model(load().qed_sampler_set, ctx, params, fallback, log10_chi_lo, log10_chi_hi)


def qed_pair_sampler_set(ctx, params=None, fallback=None, log10_chi_lo=-1.5, log10_chi_hi=2.5):
    """Install (or remove) the photon path's network of the energy split."""
    return _set_model(load().qed_pair_sampler_set, ctx, params, fallback, log10_chi_lo, log10_chi_hi)


def qed_pair_sampler_infer(ctx, chi, u, d, n):
    return load().qed_pair_sampler_infer(ctx, chi, u, d, int(n))


def qed_sampler_infer(ctx, chi, u, x, n):
    return load().qed_sampler_infer(ctx, chi, u, x, int(n))


def qed_emission_rate(ctx, chi, out, n):
    return load().qed_emission_rate(ctx, chi, out, int(n))


def qed_pair_rate(ctx, chi, out, n):
    return load().qed_pair_rate(ctx, chi, out, int(n))


def qed_gather(ctx, grid, species, out_ptrs):
    """grid: qed_grid; species: qed_species; out_ptrs: six device addresses (Ex .. Bz)."""
    return load().qed_gather(ctx, C.byref(grid), C.byref(species), (C.c_void_p * 6)(*out_ptrs))


def qed_deposit(ctx, grid, species, charge, jx, jy, jz):
    return load().qed_deposit(ctx, C.byref(grid), C.byref(species), float(charge), jx, jy, jz)


def cell_geometry(geom):
    """qed_grid holding only a geometry: dict with nx, ny, nz, x0, y0, z0, dx, dy, dz."""
    g = qed_grid()
    for k in ("nx", "ny", "nz"):
        setattr(g, k, int(geom[k]))
    for k in ("x0", "y0", "z0", "dx", "dy", "dz"):
        setattr(g, k, float(geom[k]))
    return g


def qed_substep_cells(ctx, cells):
    """cells: qed_grid, a geometry dict (cell_geometry) or None (per-particle sub-steps)."""
    if cells is None:
        return load().qed_substep_cells(ctx, None)
    if isinstance(cells, dict):
        cells = cell_geometry(cells)
    return load().qed_substep_cells(ctx, C.byref(cells))


def qed_event_gaps(ctx, hist_ptr, nbins):
    """hist_ptr: device address of 2 * nbins uint64 (or None to disable)."""
    return load().qed_event_gaps(ctx, hist_ptr, int(nbins))


def qed_emission_cdf(ctx, lo, hi, nchi, nx):
    """(cdf [nchi, nx + 1], total [nchi]) as numpy float64."""
    cdf = np.zeros((nchi, nx + 1), np.float64)
    tot = np.zeros(nchi, np.float64)
    _check(load().qed_emission_cdf(ctx, float(lo), float(hi), int(nchi), int(nx), _ptr(cdf), _ptr(tot)),
           "qed_emission_cdf")
    return cdf, tot


def qed_train_config_default():
    cfg = qed_train_config()
    _check(load().qed_train_config_default(C.byref(cfg)), "qed_train_config_default")
    return cfg


def qed_train_sampler(ctx, cfg, init=None):
    """Train on the GPU; returns (params, loss per step, CDF error per bin, fallback flags)."""
    params = np.zeros(QED_MLP_NPARAMS, np.float32)
    loss = np.zeros(cfg.steps, np.float32)
    err = np.zeros(cfg.nbins, np.float32)
    fb = np.zeros(cfg.nbins, np.uint8)
    ini = None if init is None else np.ascontiguousarray(init, np.float32)
    _check(load().qed_train_sampler(ctx, C.byref(cfg), None if ini is None else _ptr(ini), _ptr(params),
                                    _ptr(loss), _ptr(err), _ptr(fb)), "qed_train_sampler")
    return params, loss, err, fb


def qed_mlp_gradient(ctx, params, samples):
    """(loss, gradient) of the training loss from the GPU kernels."""
    p = np.ascontiguousarray(params, np.float32)
    smp = np.ascontiguousarray(samples, np.float32)
    n = smp.shape[0]
    grad = np.zeros(QED_MLP_NPARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    _check(load().qed_mlp_gradient(ctx, _ptr(p), _ptr(smp), int(n), _ptr(loss), _ptr(grad)), "qed_mlp_gradient")
    return float(loss[0]), grad


# ---------------------------------------------------------------- torch helpers

def _torch():
    import torch
    return torch


class SpeciesBuffers:
    """Device SoA buffers of one species (torch tensors) with a fixed capacity."""

    def __init__(self, capacity, real, device="cuda", parent=True, events=True, tau=False, birth=False):
        torch = _torch()
        self.capacity = int(capacity)
        self.real = real
        cap = max(1, self.capacity)
        self.n = torch.zeros(1, dtype=torch.int64, device=device)
        self.x = torch.zeros(cap, dtype=torch.float64, device=device)
        self.y = torch.zeros(cap, dtype=torch.float64, device=device)
        self.z = torch.zeros(cap, dtype=torch.float64, device=device)
        self.ux = torch.zeros(cap, dtype=real, device=device)
        self.uy = torch.zeros(cap, dtype=real, device=device)
        self.uz = torch.zeros(cap, dtype=real, device=device)
        self.w = torch.zeros(cap, dtype=real, device=device)
        self.id = torch.zeros(cap, dtype=torch.int64, device=device)
        self.parent = torch.zeros(cap, dtype=torch.int64, device=device) if parent else None
        self.events = torch.zeros(cap, dtype=torch.int32, device=device) if events else None
        self.tau = torch.full((cap,), -1.0, dtype=torch.float64, device=device) if tau else None
        self.birth = torch.zeros(cap, dtype=torch.float64, device=device) if birth else None

    def struct(self):
        s = qed_species()
        s.n = self.n.data_ptr()
        s.capacity = self.capacity
        for k in ("x", "y", "z", "ux", "uy", "uz", "w", "id"):
            setattr(s, k, getattr(self, k).data_ptr())
        s.parent = self.parent.data_ptr() if self.parent is not None else None
        s.events = self.events.data_ptr() if self.events is not None else None
        s.tau = self.tau.data_ptr() if self.tau is not None else None
        s.birth = self.birth.data_ptr() if self.birth is not None else None
        return s

    def upload(self, host):
        """host: dict of numpy arrays x,y,z,ux,uy,uz,w (float64) and id (uint64)."""
        torch = _torch()
        n = int(host["id"].size)
        if n > self.capacity:
            raise ValueError("capacity too small")
        for k in ("x", "y", "z"):
            getattr(self, k)[:n].copy_(torch.from_numpy(np.ascontiguousarray(host[k], np.float64)))
        for k in ("ux", "uy", "uz", "w"):
            getattr(self, k)[:n].copy_(torch.from_numpy(np.ascontiguousarray(host[k], np.float64)).to(self.real))
        self.id[:n].copy_(torch.from_numpy(np.ascontiguousarray(host["id"]).view(np.int64)))
        if self.parent is not None:   # uploaded particles have no parent in this run (0) unless given
            self.parent.zero_()
            if "parent" in host:
                self.parent[:n].copy_(torch.from_numpy(np.ascontiguousarray(host["parent"]).view(np.int64)))
        if self.tau is not None:
            self.tau.fill_(-1.0)
            if "tau" in host:
                self.tau[:n].copy_(torch.from_numpy(np.ascontiguousarray(host["tau"], np.float64)))
        self.n.fill_(n)

    def count(self):
        return int(self.n.item())

    def download(self):
        n = self.count()
        out = {k: getattr(self, k)[:n].double().cpu().numpy() for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
        out["id"] = self.id[:n].cpu().numpy().view(np.uint64)
        if self.parent is not None:
            out["parent"] = self.parent[:n].cpu().numpy().view(np.uint64)
        if self.tau is not None:
            out["tau"] = self.tau[:n].cpu().numpy()
        if self.birth is not None:
            out["birth"] = self.birth[:n].cpu().numpy()
        return out

    def events_host(self, n):
        return self.events[:n].cpu().numpy().astype(np.uint32)


class FieldBuffers:
    """Per-species field: either uniform (6 values) or per-slot arrays."""

    def __init__(self, host, real, device="cuda", capacity=None):
        torch = _torch()
        self.host = host
        vals = [np.asarray(host[k], np.float64).ravel() for k in ("ex", "ey", "ez", "bx", "by", "bz")]
        self.stride = 0 if vals[0].size == 1 else 1
        size = 1 if self.stride == 0 else max(int(capacity or vals[0].size), vals[0].size)
        self.t = []
        for v in vals:
            t = torch.zeros(size, dtype=real, device=device)
            t[:v.size].copy_(torch.from_numpy(v).to(real))
            self.t.append(t)

    def set_uniform(self, host):
        for t, k in zip(self.t, ("ex", "ey", "ez", "bx", "by", "bz")):
            t.fill_(float(np.asarray(host[k]).ravel()[0]))

    def struct(self):
        f = qed_field()
        for t, k in zip(self.t, ("ex", "ey", "ez", "bx", "by", "bz")):
            setattr(f, k, t.data_ptr())
        f.stride = self.stride
        return f


class Generator:
    """A context plus the three species buffers; convenience for tests and the benchmark."""

    def __init__(self, precision=QED_PREC_MIXED, capacity=(1 << 20, 1 << 20, 1 << 20), emission=True,
                 pairs=True, p_max=0.01, scheduler=QED_SCHED_NAIVE, pair_bound_coef=0.1,
                 max_substeps=1 << 24, device=0, stream=None, parent=True, events=True,
                 sampler=QED_SAMPLER_REJECTION, cascade_generations=0, surrogate_p_max=0.1,
                 pair_sampler=QED_SAMPLER_REJECTION):
        torch = _torch()
        self.real = torch.float64 if precision == QED_PREC_F64 else torch.float32
        self.precision = precision
        cfg = qed_config_default()
        cfg.device = device
        cfg.stream = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        cfg.precision = precision
        cfg.p_max = p_max
        cfg.emission = int(emission)
        cfg.pairs = int(pairs)
        cfg.scheduler = scheduler
        cfg.pair_bound_coef = pair_bound_coef
        cfg.max_substeps = max_substeps
        cfg.sampler = sampler
        cfg.cascade_generations = cascade_generations
        cfg.surrogate_p_max = surrogate_p_max
        cfg.pair_sampler = pair_sampler
        self.cfg = cfg
        self.ctx = qed_init(cfg)
        surr = sampler == QED_SAMPLER_SURROGATE
        psurr = pair_sampler == QED_SAMPLER_SURROGATE
        self.sp = [SpeciesBuffers(c, self.real, parent=parent, events=events, tau=(surr and k < 2) or (psurr and k == 2),
                                  birth=cascade_generations > 0)
                   for k, c in enumerate(capacity)]
        self.fields = [None, None, None]

    def load_state(self, state):
        for s, name in enumerate(SPECIES):
            self.sp[s].upload(state[name])

    def set_fields(self, fields, per_species=None):
        """fields: one field dict for all species, or per_species list of three."""
        fl = per_species or [fields, fields, fields]
        self.fields = [FieldBuffers(f, self.real, capacity=self.sp[s].capacity) for s, f in enumerate(fl)]

    def particles(self):
        p = qed_particles()
        for s, name in enumerate(SPECIES):
            setattr(p, name, self.sp[s].struct())
        return p

    def step(self, dt, seed, step):
        st = qed_step(self.ctx, self.particles(), [f.struct() for f in self.fields], dt, seed, step)
        _check(st, "qed_step")

    def sync(self):
        return qed_sync(self.ctx)

    def stats(self):
        return qed_get_stats(self.ctx)

    def close(self):
        if self.ctx:
            qed_finalize(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def synchrotron(ctx, x, F=None, G=None):
    """F, G of a torch device tensor x (float32 or float64)."""
    torch = _torch()
    dtype = QED_F32 if x.dtype == torch.float32 else QED_F64
    if F is None:
        F = torch.empty_like(x)
    if G is None:
        G = torch.empty_like(x)
    _check(qed_synchrotron(ctx, x.data_ptr(), F.data_ptr(), G.data_ptr(), x.numel(), dtype), "qed_synchrotron")
    return F, G
