"""qed_step_static (no allocation in the call: per-slot scratch in a static device
array) against qed_step on the same inputs: bit-identical particles and counters on
two calls in a row, the second with a smaller population, under the naive and binned
schedulers with pair creation (so the photon lists, the binned queues and the
compaction all use the static array); and the size limit."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _sorted(d):
    o = np.argsort(d["id"])
    return {k: v[o] for k, v in d.items()}


def _gen(qed, sched, cap):
    return qed.Generator(precision=qed.QED_PREC_MIXED, capacity=cap, scheduler=sched)


@pytest.mark.parametrize("sched_name", ["naive", "binned"])
def test_static_step_equals_step(sched_name):
    from paper_2008_10468_amd import qed
    sched = qed.QED_SCHED_NAIVE if sched_name == "naive" else qed.QED_SCHED_BINNED
    cap = (1 << 17, 1 << 15, 1 << 18)
    ref, sta = _gen(qed, sched, cap), _gen(qed, sched, cap)
    big = workloads.c2(n_e=60000, n_g=20000, seed=41)
    small = workloads.c2(n_e=9000, n_g=2500, seed=42)
    for call, w in enumerate((big, small)):
        print("qed_step_static:", sched_name, "call", call, "e-", w["electrons"]["id"].size, flush=True)
        for g in (ref, sta):
            g.load_state(w)
            g.set_fields(workloads.c2_field(call))
            qed.qed_reset_stats(g.ctx)
        fl = [f.struct() for f in ref.fields]
        assert qed.qed_step(ref.ctx, ref.particles(), fl, w["dt"], 3, call) == qed.QED_OK
        fl = [f.struct() for f in sta.fields]
        assert qed.qed_step_static(sta.ctx, sta.particles(), fl, w["dt"], 3, call) == qed.QED_OK
        for g in (ref, sta):
            assert g.sync()[0] == qed.QED_OK
        for s in range(3):
            a, b = _sorted(ref.sp[s].download()), _sorted(sta.sp[s].download())
            assert a["id"].size == b["id"].size, (call, s)
            for k in a:
                assert np.array_equal(a[k], b[k]), (call, s, k)
        sa, sb = ref.stats(), sta.stats()
        assert list(sa.substeps) == list(sb.substeps) and sa.emissions == sb.emissions and sa.pairs == sb.pairs
        assert sa.pairs > 0 and sa.emissions > 0
    ref.close()
    sta.close()


def test_static_step_size_limit():
    from paper_2008_10468_amd import qed
    g = qed.Generator(precision=qed.QED_PREC_MIXED, capacity=(1024, 1024, qed.QED_STATIC_MAX_SLOTS + 1))
    w = workloads.c2(n_e=512, n_g=128, seed=43)
    g.load_state(w)
    g.set_fields(workloads.c2_field(0))
    fl = [f.struct() for f in g.fields]
    assert qed.qed_step_static(g.ctx, g.particles(), fl, w["dt"], 1, 0) == qed.QED_ERR_SCRATCH
    # nothing was enqueued: the population is unchanged
    assert g.sp[0].count() == 512 and g.sp[2].count() == 128
    assert g.sync()[0] == qed.QED_OK
    g.close()
