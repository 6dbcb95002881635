"""Whole steps recorded into a HIP graph (qed_graph_*) give the eager result on
every replay, with eager work and synchronisations between the replays."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _state(g):
    out = []
    for s in range(3):
        d = g.sp[s].download()
        o = np.argsort(d["id"])
        out.append({k: v[o] for k, v in d.items() if k != "parent"})
    return out


@pytest.mark.parametrize("sched", ["naive", "binned"])
def test_graph_replays_match_eager(sched):
    from paper_2008_10468_amd import qed
    stream = torch.cuda.Stream()
    w = workloads.c2(n_e=30000, n_g=8000, seed=4)
    sc = qed.QED_SCHED_BINNED if sched == "binned" else qed.QED_SCHED_NAIVE
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 16, 1 << 15, 1 << 18), scheduler=sc,
                      stream=stream.cuda_stream)
    fields = [qed.FieldBuffers(workloads.c2_field(s), g.real) for s in range(4)]

    def steps():
        for s in range(4):
            st = qed.qed_step(g.ctx, g.particles(), [fields[s].struct()] * 3, w["dt"], 9, s)
            assert st == qed.QED_OK

    g.load_state(w)
    torch.cuda.synchronize()
    steps()
    assert g.sync()[0] == qed.QED_OK
    ref = _state(g)
    assert qed.qed_graph_begin(g.ctx) == qed.QED_OK
    assert qed.qed_sync(g.ctx)[0] == qed.QED_ERR_STATE   # no host waits while recording
    steps()
    st, graph = qed.qed_graph_end(g.ctx)
    assert st == qed.QED_OK
    for rep in range(3):
        g.load_state(w)
        torch.cuda.synchronize()
        # some eager work of the program between replays
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        assert qed.qed_graph_launch(g.ctx, graph) == qed.QED_OK
        assert g.sync()[0] == qed.QED_OK
        got = _state(g)
        for s in range(3):
            for k in ref[s]:
                assert np.array_equal(ref[s][k], got[s][k]), (rep, s, k)
    qed.qed_graph_destroy(graph)
    g.close()


def test_graph_needs_created_stream():
    from paper_2008_10468_amd import qed
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(16, 16, 16), stream=0)
    assert qed.qed_graph_begin(g.ctx) == qed.QED_ERR_STATE
    g.close()


def test_counted_steps_match_numbered_steps():
    """qed_step_counted reads the step number on the device and advances it: three
    counted steps from 5 are the steps 5, 6, 7 of qed_step, bit for bit."""
    from paper_2008_10468_amd import qed
    w = workloads.c2(n_e=20000, n_g=6000, seed=5)
    outs = []
    for counted in (False, True):
        g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 16, 1 << 15, 1 << 18))
        g.load_state(w)
        g.set_fields(workloads.c2_field(0))
        ctr = torch.full((1,), 5, dtype=torch.int32, device="cuda")
        flds = [f.struct() for f in g.fields]
        for s in range(5, 8):
            if counted:
                st = qed.qed_step_counted(g.ctx, g.particles(), flds, w["dt"], 3, ctr.data_ptr())
            else:
                st = qed.qed_step(g.ctx, g.particles(), flds, w["dt"], 3, s)
            assert st == qed.QED_OK
        assert g.sync()[0] == qed.QED_OK
        if counted:
            assert int(ctr.item()) == 8
        outs.append(_state(g))
        g.close()
    for s in range(3):
        for k in outs[0][s]:
            assert np.array_equal(outs[0][s][k], outs[1][s][k]), (s, k)
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(16, 16, 16))
    g.set_fields(workloads.c2_field(0))
    assert qed.qed_step_counted(g.ctx, g.particles(), [f.struct() for f in g.fields], 1.0, 3, None) == \
        qed.QED_ERR_INVALID_ARG
    g.close()


@pytest.mark.parametrize("sched", ["naive", "binned"])
def test_one_recorded_counted_step_replays_as_consecutive_steps(sched):
    """A graph of ONE counted step, replayed three times (eager work and host waits
    between the replays), runs steps 2, 3, 4: the same state as three eager steps."""
    from paper_2008_10468_amd import qed
    stream = torch.cuda.Stream()
    w = workloads.c2(n_e=30000, n_g=8000, seed=6)
    sc = qed.QED_SCHED_BINNED if sched == "binned" else qed.QED_SCHED_NAIVE
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 16, 1 << 15, 1 << 18), scheduler=sc,
                      stream=stream.cuda_stream)
    g.set_fields(workloads.c2_field(0))
    flds = [f.struct() for f in g.fields]
    g.load_state(w)
    torch.cuda.synchronize()
    for s in (2, 3, 4):
        assert qed.qed_step(g.ctx, g.particles(), flds, w["dt"], 11, s) == qed.QED_OK
    assert g.sync()[0] == qed.QED_OK
    ref = _state(g)
    ctr = torch.full((1,), 2, dtype=torch.int32, device="cuda")
    g.load_state(w)
    torch.cuda.synchronize()
    assert qed.qed_graph_begin(g.ctx) == qed.QED_OK
    assert qed.qed_step_counted(g.ctx, g.particles(), flds, w["dt"], 11, ctr.data_ptr()) == qed.QED_OK
    st, graph = qed.qed_graph_end(g.ctx)
    assert st == qed.QED_OK
    assert int(ctr.item()) == 2   # recording ran nothing
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        assert qed.qed_graph_launch(g.ctx, graph) == qed.QED_OK
        assert g.sync()[0] == qed.QED_OK
        assert int(ctr.item()) == 3 + rep
    got = _state(g)
    for s in range(3):
        for k in ref[s]:
            assert np.array_equal(ref[s][k], got[s][k]), (s, k)
    qed.qed_graph_destroy(graph)
    g.close()


def test_graph_replay_after_scratch_grows():
    """A recorded graph keeps the scratch addresses it was recorded with: an eager step on
    a larger population on the same context, which replaces the library's scratch with
    larger buffers, leaves the graph's replays equal to the steps it recorded."""
    from paper_2008_10468_amd import qed
    stream = torch.cuda.Stream()
    w = workloads.c2(n_e=20000, n_g=6000, seed=7)
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1 << 15, 1 << 14, 1 << 16),
                      scheduler=qed.QED_SCHED_BINNED, stream=stream.cuda_stream)
    fields = qed.FieldBuffers(workloads.c2_field(0), g.real)

    def steps(p):
        for s in range(2):
            assert qed.qed_step(g.ctx, p, [fields.struct()] * 3, w["dt"], 9, s) == qed.QED_OK

    g.load_state(w)
    torch.cuda.synchronize()
    steps(g.particles())
    assert g.sync()[0] == qed.QED_OK
    ref = _state(g)
    assert qed.qed_graph_begin(g.ctx) == qed.QED_OK
    steps(g.particles())
    st, graph = qed.qed_graph_end(g.ctx)
    assert st == qed.QED_OK
    # four times the population on the same context: photon and scheduler scratch grow
    big = [qed.SpeciesBuffers(c, g.real, parent=False, events=False) for c in (1 << 17, 1 << 16, 1 << 18)]
    w2 = workloads.c2(n_e=80000, n_g=24000, seed=8)
    pb = qed.qed_particles()
    for sb, name in zip(big, qed.SPECIES):
        sb.upload(w2[name])
        setattr(pb, name, sb.struct())
    torch.cuda.synchronize()
    steps(pb)
    assert g.sync()[0] == qed.QED_OK
    assert big[2].count() > 24000
    for rep in range(2):
        g.load_state(w)
        torch.cuda.synchronize()
        assert qed.qed_graph_launch(g.ctx, graph) == qed.QED_OK
        assert g.sync()[0] == qed.QED_OK
        got = _state(g)
        for s in range(3):
            for k in ref[s]:
                assert np.array_equal(ref[s][k], got[s][k]), (rep, s, k)
    qed.qed_graph_destroy(graph)
    g.close()
