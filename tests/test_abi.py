"""The C ABI on the host (no GPU needed): the built library loads and exports every
entry point include/qed.h declares, the Python binding names all of them and lays out
every struct exactly as a C compiler does, the host-only calls behave as documented,
and configurations are rejected before any device work."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qed.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"QED_API\s+[\w\s\*]*?\b(qed_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def qed():
    from paper_2008_10468_amd import qed as q
    if not os.path.exists(q.LIB_PATH):
        from paper_2008_10468_amd import build
        build.build()
    return q


def test_header_declares_the_entry_points():
    names = _declared()
    assert len(names) >= 30
    for must in ("qed_init", "qed_step", "qed_step_counted", "qed_sync", "qed_synchrotron", "qed_finalize",
                 "qed_get_stats", "qed_graph_begin", "qed_gather", "qed_deposit", "qed_substep_cells",
                 "qed_train_sampler", "qed_pair_sampler_set"):
        assert must in names


def test_library_exports_every_declared_symbol(qed):
    lib = C.CDLL(qed.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding covers the whole ABI
    assert sorted(set(qed.EXPORTS)) == _declared()


def test_struct_layouts_match_the_c_compiler(qed, tmp_path):
    structs = {name: getattr(qed, name) for name in
               ("qed_species", "qed_particles", "qed_field", "qed_grid", "qed_config", "qed_report", "qed_stats",
                "qed_tuning", "qed_sampler_model", "qed_train_config", "qed_kernel_time")}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qed.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} sizeof %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        name, field, value = line.split()
        cls = structs[name]
        got = C.sizeof(cls) if field == "sizeof" else getattr(cls, field).offset
        assert got == int(value), (name, field, got, value)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in structs.values())


def test_host_only_calls(qed):
    lib = qed.load()
    cfg = qed.qed_config_default()
    assert cfg.precision == qed.QED_PREC_MIXED and cfg.p_max == 0.01 and cfg.pair_bound_coef == 0.1
    assert cfg.emission == 1 and cfg.pairs == 1 and cfg.cascade_generations == 0
    assert cfg.sampler == qed.QED_SAMPLER_REJECTION and cfg.pair_sampler == qed.QED_SAMPLER_REJECTION
    tc = qed.qed_train_config_default()
    assert tc.target == 0 and tc.nbins > 0 and tc.tolerance > 0
    assert lib.qed_config_default(None) == qed.QED_ERR_INVALID_ARG
    for st in (qed.QED_OK, qed.QED_ERR_INVALID_ARG, qed.QED_ERR_CAPACITY, qed.QED_ERR_NONFINITE, qed.QED_ERR_HIP,
               qed.QED_ERR_STATE):
        assert lib.qed_status_string(st)


def test_bad_configurations_are_rejected_before_device_work(qed):
    """qed_init validates the configuration before it touches the HIP runtime, so these
    are rejected here, without a GPU."""
    lib = qed.load()
    base = qed.qed_config_default()

    def rejected(**kw):
        cfg = qed.qed_config_default()
        for k, v in kw.items():
            setattr(cfg, k, v)
        ctx = C.c_void_p()
        return lib.qed_init(C.byref(ctx), C.byref(cfg)) == qed.QED_ERR_INVALID_ARG and not ctx.value

    assert rejected(precision=7)
    assert rejected(p_max=0.0) and rejected(p_max=1.5) and rejected(p_max=float("nan"))
    assert rejected(pair_bound_coef=-1.0)
    assert rejected(max_substeps=0)
    assert rejected(scheduler=9)
    assert rejected(sampler=qed.QED_SAMPLER_SURROGATE, precision=qed.QED_PREC_F64)
    assert rejected(cascade_generations=65)
    assert rejected(cascade_generations=2, sampler=qed.QED_SAMPLER_SURROGATE)
    assert rejected(pair_sampler=qed.QED_SAMPLER_SURROGATE, cascade_generations=1)
    assert lib.qed_init(None, C.byref(base)) == qed.QED_ERR_INVALID_ARG


def test_bench_reads_traffic_only_for_the_kernels_as_they_stand(tmp_path, monkeypatch):
    """bench.py reports a measured traffic figure only for the run and step count it was
    taken over, and only while the kernel sources hash to the value recorded beside it."""
    import bench
    sha = bench.kernel_source_hash()
    assert re.fullmatch(r"[0-9a-f]{64}", sha) and sha == bench.kernel_source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: sha)
    (prof / "hbm_traffic_hotspot.md").write_text(
        f"source_sha256: {sha}\nsteps: 20\ntraffic plain_binned k_heavy 123456\ntraffic surrogate_binned k_heavy 654321\n")
    assert bench.measured_traffic("k_heavy", "hotspot", "plain_binned", 20) == 123456.0
    assert bench.measured_traffic("k_heavy", "hotspot", "surrogate_binned", 20) == 654321.0
    assert bench.measured_traffic("k_heavy", "hotspot", "plain_binned", 8) is None     # other step count
    assert bench.measured_traffic("k_lepton", "hotspot", "plain_binned", 20) is None
    assert bench.measured_traffic("k_heavy", "c3", "plain_binned", 20) is None
    (prof / "hbm_traffic_hotspot.md").write_text("source_sha256: " + "0" * 64 + "\nsteps: 20\n"
                                                 "traffic plain_binned k_heavy 123456\n")
    assert bench.measured_traffic("k_heavy", "hotspot", "plain_binned", 20) is None
