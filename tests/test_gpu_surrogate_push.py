"""The push of the lepton optical-depth path against the oracle's Boris push.

In a pure magnetic field the optical-depth path advances a lepton through all the
sub-steps up to its next emission (or the end of the step) at once, in closed form
(rotate_many: the m-fold Boris rotation as a power of e^{i theta}, and the sum of the
moves as a geometric series).  Leptons given an optical depth far above what a step
can use do not emit, so their end-of-step momentum and position must be those of the
path's N Boris sub-steps of Algorithm 1 (push, then move by u sub_t / gamma), which
the oracle takes one by one in FP64 from the same float start values.  The field is
along a direction off the axes, both charges are present, N runs from 1 (the single
sub-step, which the path takes as the loop body) to several thousand, and the turn
per sub-step from about 1e-3 to nearly pi."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _population(n, seed, bdir):
    rng = np.random.default_rng(seed)
    gamma = 10.0 ** rng.uniform(1.0, 4.0, n)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    # one in twenty nearly along B: chi close to zero, a single sub-step
    few = rng.random(n) < 0.05
    d[few] = bdir + 1e-7 * d[few]
    d /= np.linalg.norm(d, axis=1)[:, None]
    u = (np.sqrt(gamma ** 2 - 1.0)[:, None] * d).astype(np.float32)
    pos = rng.uniform(-1e4, 1e4, (n, 3))
    sp = {"x": pos[:, 0], "y": pos[:, 1], "z": pos[:, 2], "ux": u[:, 0], "uy": u[:, 1], "uz": u[:, 2],
          "w": np.ones(n, np.float32), "id": np.arange(1, n + 1, dtype=np.uint64) + np.uint64(seed << 40),
          "tau": np.full(n, 1e300)}
    return sp


@pytest.mark.parametrize("n, dt, nmax", [(1000, 1.0e6, 100), (64, 3.0e7, 4096)])
@pytest.mark.parametrize("scheduler", ["naive", "binned"])
def test_closed_form_push_matches_oracle_boris(scheduler, n, dt, nmax):
    """(1000 leptons per species, N up to 225) and (64, N up to 6718: 13 bits of binary
    powering)."""
    from paper_2008_10468_amd import qed
    bdir = np.array([0.36, -0.48, 0.8])
    B = 2e-3 * bdir
    p_s = 0.1
    sched = {"naive": qed.QED_SCHED_NAIVE, "binned": qed.QED_SCHED_BINNED}[scheduler]
    el, po = _population(n, 31, bdir), _population(n, 32, bdir)
    emp = {k: np.zeros(0) for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
    emp["id"] = np.zeros(0, np.uint64)
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(n, n, 16), pairs=False,
                      sampler=qed.QED_SAMPLER_SURROGATE, surrogate_p_max=p_s, scheduler=sched)
    g.load_state({"electrons": el, "positrons": po, "photons": emp})
    g.set_fields(workloads.uniform_field(bx=B[0], by=B[1], bz=B[2]))
    g.step(dt, 5, 0)
    st, rep = g.sync()
    assert st == qed.QED_OK
    stats = g.stats()
    assert stats.emissions == 0
    out = [g.sp[0].download(), g.sp[1].download()]
    g.close()
    Bv = np.asarray(B, np.float64)
    zero = np.zeros(3)
    ns = []
    for s, (src, q) in enumerate(((el, -1.0), (po, 1.0))):
        got = out[s]
        order = np.argsort(got["id"])
        got = {k: v[order] for k, v in got.items()}
        assert np.array_equal(got["id"], src["id"])
        for i in range(n):
            u = np.array([src["ux"][i], src["uy"][i], src["uz"][i]], np.float64)
            gam = np.sqrt(1.0 + u @ u)
            chi = oracle.chi_lepton(u, zero, Bv)
            N = oracle.nsub(oracle.bound_emission(chi, gam, dt), p_s)
            ns.append(N)
            sub = dt / N
            x = np.array([src["x"][i], src["y"][i], src["z"][i]])
            path = 0.0
            for _ in range(N):
                u = oracle.boris(u, zero, Bv, q, sub)
                v = u * (sub / np.sqrt(1.0 + u @ u))
                x = x + v
                path += np.linalg.norm(v)
            ug = np.array([got["ux"][i], got["uy"][i], got["uz"][i]], np.float64)
            xg = np.array([got["x"][i], got["y"][i], got["z"][i]])
            # Float rotation vectors: t = q B sub_t / (2 gamma) carries a relative error of a
            # few float roundings (up to about 3e-7 with the hardware reciprocal square
            # root), so each sub-step turns by theta (1 + O(3e-7)) and the phase drifts by up
            # to that fraction of the total turn N theta, in the path's sub-step loop as in
            # closed form (whose powering runs in double); on top of that a few roundings of
            # |u| and of the path length.
            turn = N * 2.0 * np.arctan(np.linalg.norm(Bv) * sub / (2.0 * gam))
            tol = 4e-6 + 5e-7 * turn
            assert np.linalg.norm(ug - u) <= tol * np.linalg.norm(u), (s, i, N, turn, ug, u)
            assert np.linalg.norm(xg - x) <= tol * path + 1e-9 * np.linalg.norm(x), (s, i, N, turn, xg, x)
    ns = np.array(ns)
    assert ns.min() == 1 and ns.max() >= nmax and (ns >= 2).mean() > 0.9
