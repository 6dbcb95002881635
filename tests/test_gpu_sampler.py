"""The surrogate sampler on the GPU: the total-rate fit, the CDF table, the
training kernels' gradients and the trained network against the oracle, and the
surrogate generator's statistics against the exact emission law.

The surrogate is statistically equivalent to Algorithm 1, not particle by
particle: its tests compare distributions at 3 sigma."""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import mlp_ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALPHA = 7.2973525693e-3


def _ctx():
    from paper_2008_10468_amd import qed
    return qed, qed.qed_init(qed.qed_config_default())


def _h_oracle(chi):
    """chi q(chi) = gamma / (alpha dt) * int_0^1 P_m dx (the exact total rate)."""
    return oracle.emission_prob(float(chi), 1.0, 1.0, False) / ALPHA


def test_rate_fit_matches_oracle():
    qed, ctx = _ctx()
    chi = np.float32(10.0) ** np.linspace(-6, 4.7, 120).astype(np.float32)
    d = torch.from_numpy(chi).cuda()
    out = torch.empty_like(d)
    assert qed.qed_emission_rate(ctx, d.data_ptr(), out.data_ptr(), chi.size) == qed.QED_OK
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = np.array([_h_oracle(c) for c in chi.astype(np.float64)])
    err = np.abs(got / ref - 1)
    assert err.max() <= 1e-6, (chi[np.argmax(err)], err.max())
    # zero and tiny chi
    z = torch.tensor([0.0, 1e-30], device="cuda")
    o = torch.empty_like(z)
    assert qed.qed_emission_rate(ctx, z.data_ptr(), o.data_ptr(), 2) == qed.QED_OK
    assert o[0].item() == 0.0 and abs(o[1].item() / (1e-30 * 5 * math.sqrt(3) / 6) - 1) < 1e-6
    qed.qed_finalize(ctx)


def test_cdf_table_matches_oracle():
    qed, ctx = _ctx()
    nchi, nx = 11, 4096
    cdf, tot = qed.qed_emission_cdf(ctx, -3.0, 2.0, nchi, nx)
    xi = np.arange(nx + 1) / nx
    xg = 1.0 - (1.0 - xi) ** 2
    assert np.all(np.diff(cdf, axis=1) >= -1e-14) and np.all(cdf[:, 0] == 0) and np.all(cdf[:, -1] == 1)
    for c in range(0, nchi, 2):
        chi = 10.0 ** (-3.0 + 0.5 * c)
        b = 1.5 * chi
        # total: int_0^1 P_m / (c b) with c = sqrt(3) alpha / pi at gamma = dt = 1
        ref_tot = oracle.emission_prob(chi, 1.0, 1.0, False) * math.pi / (math.sqrt(3) * ALPHA * b)
        assert abs(tot[c] / ref_tot - 1) <= 2e-6, (chi, tot[c], ref_tot)
        for k in np.linspace(1, nx - 1, 9).astype(int):
            ref = oracle.emission_cdf(chi, xg[k] ** 3)
            assert abs(cdf[c, k] - ref) <= 2e-6, (chi, xg[k], cdf[c, k], ref)
    qed.qed_finalize(ctx)


def test_mlp_gradient_matches_reference():
    qed, ctx = _ctx()
    rng = np.random.default_rng(5)
    p = np.zeros(mlp_ref.NPARAMS)
    for name, (fin, fout) in {"W1": (2, 64), "W2": (64, 64), "W3": (64, 64), "W4": (64, 1)}.items():
        off = mlp_ref.OFF[name]
        size = fin * fout
        p[off:off + size] = rng.uniform(-1, 1, size) * math.sqrt(6.0 / (fin + fout))
    for name in ("b1", "b2", "b3"):
        p[mlp_ref.OFF[name]:mlp_ref.OFF[name] + 64] = rng.normal(0, 0.1, 64)
    p[mlp_ref.OFF["b4"]] = 0.3
    p = p.astype(np.float32).astype(np.float64)
    n = 2048
    smp = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(0, 2, n),
                    rng.uniform(0.1, 2.0, n)], axis=1).astype(np.float32)
    loss, grad = qed.qed_mlp_gradient(ctx, p, smp)
    # against the plain FP64 network (no rounding mirrored): loss and every tensor's
    # gradient within 1e-2 (the bfloat16 matrix-core layers are the only difference)
    L0, g0 = mlp_ref.gradient(p, smp.astype(np.float64), round_bf16=False)
    sizes = {"W1": 128, "b1": 64, "W2": 4096, "b2": 64, "W3": 4096, "b3": 64, "W4": 64, "b4": 1}
    errs = {}
    for name, off in mlp_ref.OFF.items():
        a, r = grad[off:off + sizes[name]], g0[off:off + sizes[name]]
        errs[name] = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
    print("gradient relative error per tensor against the unrounded network:", errs, "loss", loss / L0 - 1,
          flush=True)
    assert abs(loss / L0 - 1) <= 2e-3, (loss, L0)
    assert max(errs.values()) <= 1e-2, errs
    qed.qed_finalize(ctx)


@pytest.fixture(scope="module")
def trained():
    """A shorter training run on the GPU (the default run is the benchmark's)."""
    from paper_2008_10468_amd import qed
    ctx = qed.qed_init(qed.qed_config_default())
    cfg = qed.qed_train_config_default()
    cfg.steps = 40000
    params, loss, err, fb = qed.qed_train_sampler(ctx, cfg)
    qed.qed_finalize(ctx)
    return cfg, params, loss, err, fb


def test_training_is_deterministic():
    """Two short training runs give the same parameters bit for bit (fixed-order sums)."""
    from paper_2008_10468_amd import qed
    ctx = qed.qed_init(qed.qed_config_default())
    cfg = qed.qed_train_config_default()
    cfg.steps = 500
    a = qed.qed_train_sampler(ctx, cfg)
    b = qed.qed_train_sampler(ctx, cfg)
    qed.qed_finalize(ctx)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_training_reduces_loss(trained):
    cfg, params, loss, err, fb = trained
    assert np.all(np.isfinite(loss)) and np.all(np.isfinite(params))
    assert loss[-50:].mean() < 0.05 * loss[:5].mean(), (loss[:5], loss[-50:].mean())
    assert np.all(np.isfinite(err)) and err.max() < 0.5
    # nearly all of the range is learnt to the tolerance already in this shorter run
    assert np.mean(err <= cfg.tolerance) >= 0.8, err
    assert err.max() <= 3 * cfg.tolerance, err


def test_trained_network_against_oracle_cdf(trained):
    """Where the network is used, |CDF_chi(x(chi, u)^3) - u| stays within the bin's
    validated error (plus the table's own error) by the oracle's quadrature."""
    from paper_2008_10468_amd import qed
    cfg, params, loss, err, fb = trained
    ctx = qed.qed_init(qed.qed_config_default())
    assert qed.qed_sampler_set(ctx, params, fb, cfg.log10_chi_lo, cfg.log10_chi_hi) == qed.QED_OK
    rng = np.random.default_rng(11)
    n = 256
    l10 = rng.uniform(cfg.log10_chi_lo, cfg.log10_chi_hi, n)
    chi = (10.0 ** l10).astype(np.float32)
    u = rng.uniform(0, 1, n).astype(np.float32)
    dc, du = torch.from_numpy(chi).cuda(), torch.from_numpy(u).cuda()
    dx = torch.empty_like(dc)
    assert qed.qed_sampler_infer(ctx, dc.data_ptr(), du.data_ptr(), dx.data_ptr(), n) == qed.QED_OK
    torch.cuda.synchronize()
    x = dx.cpu().numpy().astype(np.float64)
    binw = (cfg.log10_chi_hi - cfg.log10_chi_lo) / cfg.nbins
    bins = np.minimum(((np.log10(chi.astype(np.float64)) - cfg.log10_chi_lo) / binw).astype(int), cfg.nbins - 1)
    used = fb[bins] == 0
    assert np.array_equal(np.isnan(x), ~used)
    checked = 0
    for k in np.flatnonzero(used)[:120]:
        c = oracle.emission_cdf(float(chi[k]), x[k] ** 3)
        assert abs(c - u[k]) <= err[bins[k]] + 2e-4, (chi[k], u[k], x[k], c, err[bins[k]])
        checked += 1
    assert checked >= 20
    qed.qed_finalize(ctx)


def _pure_b_population(n, chi, gamma, seed, id0=0):
    """n electrons with the same gamma, moving along x in B along z (chi = gamma B)."""
    u = math.sqrt(gamma * gamma - 1)
    e = {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n), "ux": np.full(n, u), "uy": np.zeros(n),
         "uz": np.zeros(n), "w": np.ones(n), "id": np.arange(id0, id0 + n, dtype=np.uint64)}
    return e, {"bz": chi / u}


def _run_surrogate(qed, n, chi, gamma, dt, model=None, seed=7, scheduler=None, p_s=0.1, photons=4,
                   sampler=None):
    e, f = _pure_b_population(n, chi, gamma, seed)
    emp = {k: np.zeros(0) for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
    emp["id"] = np.zeros(0, np.uint64)
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, 16, photons * n), pairs=False,
                      sampler=qed.QED_SAMPLER_SURROGATE if sampler is None else sampler, surrogate_p_max=p_s,
                      scheduler=qed.QED_SCHED_NAIVE if scheduler is None else scheduler)
    if model is not None:
        cfg, params, fb = model
        assert qed.qed_sampler_set(g.ctx, params, fb, cfg.log10_chi_lo, cfg.log10_chi_hi) == qed.QED_OK
    g.load_state({"electrons": e, "positrons": emp, "photons": emp})
    g.set_fields(workloads.uniform_field(**f))
    g.step(dt, seed, 0)
    st, rep = g.sync()
    assert st == qed.QED_OK
    ev = g.sp[0].events_host(n)
    ph = g.sp[2].download()
    stats = g.stats()
    g.close()
    return ev, ph, stats


@pytest.mark.parametrize("chi", [0.05, 0.7, 6.0])
@pytest.mark.parametrize("use_model", [False, True])
def test_surrogate_emission_law(trained, chi, use_model):
    """Pure B field: chi and gamma are constant until the first emission, so
    P(no emission in the step) = exp(-alpha chi q(chi) dt / gamma) exactly; the
    first photon's energy fraction follows the normalised eq. (1)."""
    from paper_2008_10468_amd import qed
    cfg, params, loss, err, fb = trained
    gamma, n = 2000.0, 200_000
    p_exact = oracle.emission_prob(chi, gamma, 1.0, False)     # per unit dt
    dt = 0.7 / p_exact
    ev, ph, stats = _run_surrogate(qed, n, chi, gamma, dt, model=(cfg, params, fb) if use_model else None)
    p0 = math.exp(-0.7)
    frac0 = float(np.mean(ev == 0))
    sig = math.sqrt(p0 * (1 - p0) / n)
    assert abs(frac0 - p0) <= 3.5 * sig, (frac0, p0, sig)
    # spectrum of the first photon of each parent (parent gamma still the initial one)
    first = {}
    for j in range(ph["id"].size):
        par = int(ph["parent"][j])
        if par not in first:
            first[par] = j
    sel = np.array(sorted(first.values()))
    # order of appends inside a parent is by sub-step: take the smallest-energy-ordering-free
    # quantity: the photon emitted first is the one with the smallest sub-step index, and the
    # parent's gamma before it is the initial gamma
    delta = np.sqrt(ph["ux"][sel] ** 2 + ph["uy"][sel] ** 2 + ph["uz"][sel] ** 2) / gamma
    m = delta.size
    for q in (0.05, 0.2, 0.4, 0.6, 0.8, 0.95):
        dq = np.quantile(delta, q)
        c = oracle.emission_cdf(chi, dq)
        s = math.sqrt(q * (1 - q) / m)
        assert abs(c - q) <= 4 * s + 2e-3, (chi, q, c, s)
    if use_model and chi >= 10 ** cfg.log10_chi_lo:
        assert stats.learned_events + stats.fallback_events == stats.emissions
    if not use_model:
        assert stats.learned_events == 0 and stats.fallback_events == stats.emissions


@pytest.mark.parametrize("flagged", ["above", "at_and_below"])
def test_fallback_flags_choose_the_sampler(trained, flagged):
    """The per-bin fallback flags pick the sampler by the chi at the emission.  In a pure B
    field chi stays constant between emissions and only falls at them (recoil).  With the
    bins above the start chi flagged, every energy comes from the network.  With the start
    chi's bin and all below flagged, every energy comes from rejection.  Either way the
    first photons' energy fractions follow the normalised eq. (1)."""
    from paper_2008_10468_amd import qed
    cfg, params, loss, err, fb0 = trained
    nb = int(np.asarray(fb0).size)
    binw = (cfg.log10_chi_hi - cfg.log10_chi_lo) / nb
    b0 = int((math.log10(0.7) - cfg.log10_chi_lo) / binw)
    chi = 10.0 ** (cfg.log10_chi_lo + (b0 + 0.5) * binw)     # the middle of its bin
    fb = np.zeros(nb, np.uint8)
    if flagged == "above":
        fb[b0 + 1:] = 1
    else:
        fb[:b0 + 1] = 1
    gamma, n = 2000.0, 50_000
    dt = 0.7 / oracle.emission_prob(chi, gamma, 1.0, False)
    ev, ph, stats = _run_surrogate(qed, n, chi, gamma, dt, model=(cfg, params, fb))
    assert stats.emissions == ph["id"].size and stats.emissions > 0.4 * n
    if flagged == "above":
        assert stats.learned_events == stats.emissions and stats.fallback_events == 0
    else:
        assert stats.learned_events == 0 and stats.fallback_events == stats.emissions
        assert stats.fallback_draws >= stats.emissions
    first = {}
    for j in range(ph["id"].size):
        first.setdefault(int(ph["parent"][j]), j)
    sel = np.array(sorted(first.values()))
    delta = np.sqrt(ph["ux"][sel] ** 2 + ph["uy"][sel] ** 2 + ph["uz"][sel] ** 2) / gamma
    for q in (0.05, 0.2, 0.5, 0.8, 0.95):
        c = oracle.emission_cdf(chi, np.quantile(delta, q))
        s = math.sqrt(q * (1 - q) / delta.size)
        assert abs(c - q) <= 4 * s + 2e-3, (flagged, q, c, s)


@pytest.mark.parametrize("p_s", [0.01, 0.1, 0.3])
def test_surrogate_event_count_is_poisson(p_s):
    """chi = 0.02 in a pure B field: the rate alpha chi q(chi) / gamma = alpha B q(chi) changes
    by well under 0.1% over the step (the recoil lowers chi by a few per cent and q is flat at
    small chi), so the number of emissions in a step is Poisson with mean W dt = 3, whatever
    the sub-step bound; dropping the optical depth's overshoot at each event would lower the
    mean by about p_s / 2 per event."""
    from paper_2008_10468_amd import qed
    chi, gamma, n, lam = 0.02, 2000.0, 200_000, 3.0
    dt = lam / oracle.emission_prob(chi, gamma, 1.0, False)
    ev, ph, stats = _run_surrogate(qed, n, chi, gamma, dt, p_s=p_s, photons=6)
    ev = ev.astype(np.float64)
    sig = math.sqrt(lam / n)
    assert abs(ev.mean() - lam) <= 4 * sig + 2e-3 * lam, (p_s, ev.mean(), sig)
    assert abs(ev.var() / lam - 1.0) <= 0.02, (p_s, ev.var())
    for k in range(8):
        pk = math.exp(-lam) * lam ** k / math.factorial(k)
        fk = float(np.mean(ev == k))
        assert abs(fk - pk) <= 4 * math.sqrt(pk * (1 - pk) / n) + 1e-3 * pk, (p_s, k, fk, pk)
    # the sub-step count follows the bound's target
    assert stats.substeps[0] < n * math.ceil(lam * 4 / p_s)


@pytest.mark.parametrize("p_s", [0.1, 0.3])
def test_surrogate_event_count_matches_plain_with_recoil(p_s):
    """chi = 1: an emission takes a large share of the energy and raises the rate per unit
    time (q grows as chi falls), so the part of a sub-step after a crossing must count at
    the rate after the recoil.  The mean number of emissions per step agrees with the
    paper's generator (Algorithm 1, p_max = 0.01) on the same population."""
    from paper_2008_10468_amd import qed
    chi, gamma, n = 1.0, 2000.0, 200_000
    dt = 3.0 / oracle.emission_prob(chi, gamma, 1.0, False)
    ev_s, _, _ = _run_surrogate(qed, n, chi, gamma, dt, p_s=p_s, photons=8)
    ev_p, _, _ = _run_surrogate(qed, n, chi, gamma, dt, photons=8, sampler=qed.QED_SAMPLER_REJECTION)
    ms, mp = ev_s.mean(), ev_p.mean()
    sig = math.sqrt(ev_s.var() / n + ev_p.var() / n)
    assert abs(ms - mp) <= 4 * sig, (p_s, ms, mp, sig)


def test_sampler_infer_ragged_sizes(trained):
    """qed_sampler_infer on 1, 17 and 333 inputs (partial 16-row passes and a partial
    wave): every row gives the value it gives inside a full batch, bit for bit."""
    from paper_2008_10468_amd import qed
    cfg, params, loss, err, fb = trained
    ctx = qed.qed_init(qed.qed_config_default())
    assert qed.qed_sampler_set(ctx, params, fb, cfg.log10_chi_lo, cfg.log10_chi_hi) == qed.QED_OK
    rng = np.random.default_rng(13)
    n = 333
    chi = (10.0 ** rng.uniform(cfg.log10_chi_lo, cfg.log10_chi_hi, n)).astype(np.float32)
    u = rng.uniform(0, 1, n).astype(np.float32)
    dc, du = torch.from_numpy(chi).cuda(), torch.from_numpy(u).cuda()
    full = torch.full_like(dc, -7.0)
    assert qed.qed_sampler_infer(ctx, dc.data_ptr(), du.data_ptr(), full.data_ptr(), n) == qed.QED_OK
    for k in (1, 17, 333):
        part = torch.full_like(dc, -7.0)
        assert qed.qed_sampler_infer(ctx, dc[-k:].data_ptr(), du[-k:].data_ptr(), part.data_ptr(), k) == qed.QED_OK
        torch.cuda.synchronize()
        a = full[-k:].cpu().numpy()
        b = part[:k].cpu().numpy()
        assert np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)]), k
        assert np.all(part[k:].cpu().numpy() == -7.0)        # nothing written past n
    qed.qed_finalize(ctx)


def test_surrogate_binned_equals_naive(trained):
    from paper_2008_10468_amd import qed
    cfg, params, loss, err, fb = trained
    w = workloads.c2(n_e=20000, n_g=5000, seed=3)
    outs = []
    for sched in (qed.QED_SCHED_NAIVE, qed.QED_SCHED_BINNED):
        g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 16, 1 << 15, 1 << 17), scheduler=sched,
                          sampler=qed.QED_SAMPLER_SURROGATE)
        assert qed.qed_sampler_set(g.ctx, params, fb, cfg.log10_chi_lo, cfg.log10_chi_hi) == qed.QED_OK
        g.load_state(w)
        for s in range(3):
            g.set_fields(workloads.c2_field(s))
            g.step(w["dt"], 5, s)
            assert g.sync()[0] == qed.QED_OK
        res = []
        for k in range(3):
            d = g.sp[k].download()
            o = np.argsort(d["id"])
            res.append({kk: v[o] for kk, v in d.items()})
        outs.append(res)
        g.close()
    a, b = outs
    for s in range(3):
        for k in a[s]:
            assert np.array_equal(a[s][k], b[s][k]), (s, k)
    # new pairs carry tau = -1 or a drawn positive value after their first step
    assert np.all((a[0]["tau"] == -1.0) | (a[0]["tau"] > 0.0))


def test_surrogate_rejects_bad_configuration():
    from paper_2008_10468_amd import qed
    cfg = qed.qed_config_default()
    cfg.sampler = qed.QED_SAMPLER_SURROGATE
    cfg.precision = qed.QED_PREC_F64
    import ctypes as C
    ctx = C.c_void_p()
    assert qed.load().qed_init(C.byref(ctx), C.byref(cfg)) == qed.QED_ERR_INVALID_ARG
    cfg.precision = qed.QED_PREC_MIXED
    for bad in (0.0, 1.5, float("nan")):
        cfg.surrogate_p_max = bad
        assert qed.load().qed_init(C.byref(ctx), C.byref(cfg)) == qed.QED_ERR_INVALID_ARG
    # the optical depth is required
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(16, 16, 16), sampler=qed.QED_SAMPLER_SURROGATE)
    g.sp[0].tau = None
    g.set_fields(workloads.uniform_field(bz=1e-3))
    assert qed.qed_step(g.ctx, g.particles(), [f.struct() for f in g.fields], 1.0, 1, 0) == qed.QED_ERR_INVALID_ARG
    # models with a bad range or bin count are refused
    p = np.zeros(qed.QED_MLP_NPARAMS, np.float32)
    assert qed.qed_sampler_set(g.ctx, p, np.zeros(0, np.uint8)) == qed.QED_ERR_INVALID_ARG
    assert qed.qed_sampler_set(g.ctx, p, np.zeros(4, np.uint8), 2.0, 1.0) == qed.QED_ERR_INVALID_ARG
    g.close()
