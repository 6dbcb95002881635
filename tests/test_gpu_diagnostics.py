"""Diagnostics (Fig. 1 event gaps, P_max sensitivity, FP64 vs mixed precision) on the
GPU: the event-gap histogram equals the oracle's, exactly on the FP64 path; the event
statistics do not depend on P_max and agree between the two precisions."""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import as_precision, oracle_step

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _state(w):
    return {s: w[s] for s in ("electrons", "positrons", "photons")}


@pytest.mark.parametrize("prec_name", ["F64", "MIXED"])
def test_event_gaps_match_oracle(prec_name):
    """C2 population (emission and pairs), three steps: the GPU's histogram of events by
    sub-steps since the particle's previous event equals the oracle's (FP64: exactly;
    mixed: up to the rare events whose decision float rounding flips)."""
    from paper_2008_10468_amd import qed
    prec = getattr(qed, "QED_PREC_" + prec_name)
    w = workloads.c2(n_e=20000, n_g=5000, seed=7)
    nb = 24
    g = qed.Generator(precision=prec, capacity=(1 << 16, 1 << 15, 1 << 17))
    g.load_state(_state(w))
    g.set_fields(w["fields"])
    hist = torch.zeros(2 * nb, dtype=torch.int64, device="cuda")
    assert qed.qed_event_gaps(g.ctx, hist.data_ptr(), nb) == qed.QED_OK
    he = np.zeros(nb, np.int64)
    hp = np.zeros(nb, np.int64)
    fh = [as_precision(f.host, prec) for f in g.fields]
    for step in range(3):
        before = [g.sp[s].download() for s in range(3)]
        print(f"event gaps: {prec_name} step {step}", flush=True)
        g.step(w["dt"], 4, step)
        assert g.sync()[0] == qed.QED_OK
        res = oracle_step(before, fh, w["dt"], 4, step, prec)
        e, p = oracle.event_gaps([res["electron"][1], res["positron"][1]], res["photon"][1], nb)
        he += e
        hp += p
    got = hist.cpu().numpy().reshape(2, nb)
    st = g.stats()
    g.close()
    assert got[0].sum() == st.emissions and got[1].sum() == st.pairs
    assert he.sum() > 500 and hp.sum() > 5
    if prec_name == "F64":
        assert np.array_equal(got[0], he) and np.array_equal(got[1], hp)
    else:
        assert np.abs(got[0] - he).sum() <= 2e-3 * he.sum() + 4
        assert np.abs(got[1] - hp).sum() <= 2e-3 * hp.sum() + 4


def test_disabling_event_gaps():
    from paper_2008_10468_amd import qed
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(16, 16, 16))
    hist = torch.zeros(2, dtype=torch.int64, device="cuda")
    assert qed.qed_event_gaps(g.ctx, hist.data_ptr(), 1) == qed.QED_ERR_INVALID_ARG
    assert qed.qed_event_gaps(g.ctx, None, 0) == qed.QED_OK
    g.close()


def test_pmax_sensitivity():
    """The C1 population (pure B): emissions agree across P_max = 0.003 .. 0.1 within
    statistics while the sub-steps scale like 1/P_max."""
    from paper_2008_10468_amd import diagnostics
    w = workloads.c1(n=16384)
    r = diagnostics.pmax_sensitivity(_state(w), w["fields"], w["dt"], 2, p_values=(0.003, 0.01, 0.03, 0.1),
                                     pairs=False)["rows"]
    ref = r[1]["emissions"]
    assert ref > 5000
    for row in r:
        assert abs(row["emissions"] - ref) <= 4 * math.sqrt(2 * ref) + 0.01 * ref, (row, ref)
        sem = math.hypot(row["photon_energy_sem"], r[1]["photon_energy_sem"])
        assert abs(row["mean_photon_energy"] - r[1]["mean_photon_energy"]) <= 4 * sem, (row, sem)
    ratio = r[0]["lepton_substeps"] / r[2]["lepton_substeps"]
    assert 8.0 < ratio < 10.5, ratio


def test_fp64_and_mixed_agree():
    """Sec. 1 and 3.2: single-precision accuracy of the synchrotron functions gives almost
    identical results.  On a C2 population the two precisions emit and create pairs at the
    same rates within statistics, with the same photon spectrum (they draw different
    random numbers, so the comparison is statistical)."""
    from paper_2008_10468_amd import diagnostics
    w = workloads.c2(n_e=100000, n_g=25000, seed=8)
    r = diagnostics.precision_comparison(_state(w), w["fields"], w["dt"], 3)
    a, b = r["f64"], r["mixed"]
    for k in ("emissions", "pairs"):
        assert abs(a[k] - b[k]) <= 4 * math.sqrt(a[k] + b[k]) + 5, (k, a[k], b[k])
    # the photon spectra span six decades: compare the distributions (two-sample KS)
    from scipy import stats as sps
    assert sps.ks_2samp(a["photon_energies"], b["photon_energies"]).pvalue > 1e-3


def test_cell_comparison():
    """Sub-steps per cell against per particle on a C2 population: the same emission and
    pair rates and photon energies within statistics, at a cost that grows with the
    particles per cell (a cell takes its particles' largest count)."""
    from paper_2008_10468_amd import diagnostics
    w = workloads.c2(n_e=100000, n_g=25000, seed=9)
    r = diagnostics.cell_comparison(_state(w), w["fields"], w["dt"], 3, cells=(None, 16, 4))["rows"]
    ref = r[0]
    assert ref["cells_per_axis"] is None and ref["emissions"] > 2000
    for row in r[1:]:
        for k in ("emissions", "pairs"):
            assert abs(row[k] - ref[k]) <= 4 * math.sqrt(row[k] + ref[k]) + 0.01 * ref[k] + 5, (k, row, ref)
        sem = math.hypot(row["photon_energy_sem"], ref["photon_energy_sem"])
        assert abs(row["mean_photon_energy"] - ref["mean_photon_energy"]) <= 4 * sem, (row, sem)
    subs = [row["lepton_substeps"] for row in r]
    assert subs[0] < subs[1] < subs[2], subs
