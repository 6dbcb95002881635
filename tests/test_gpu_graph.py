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
