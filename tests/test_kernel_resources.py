"""Register, LDS and occupancy figures of the hot kernels, as the compiler's resource
report for gfx950 gives them (host only: a device-only compile of the kernel source
with the library's own flags).  The launch shapes and the measured rates rest on them:
the photon pass holds 4 waves per SIMD (127 VGPRs, 35 KB of LDS per block), the
naive lepton pass and the heavy queue 3 and 4, the optical-depth heavy queue 2 (its
LDS: the network, the rate table and 128-entry child buffers), and no kernel uses
scratch memory (register spills to memory)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def usage(tmp_path_factory):
    from paper_2008_10468_amd import build
    try:
        cc = build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("ru") / "k.o"
    cmd = [cc, *build.FLAGS, "--cuda-device-only", "-c", os.path.join(build.CSRC, "qed_kernels.hip"), "-o", str(out),
           "-Rpass-analysis=kernel-resource-usage"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    figures = {}
    for block in re.split(r"remark: Function Name: ", res.stderr)[1:]:
        name = block.split()[0]
        f = {}
        for key, pat in (("vgpr", r"VGPRs: (\d+)"), ("occ", r"Occupancy \[waves/SIMD\]: (\d+)"),
                         ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"), ("lds", r"LDS Size \[bytes/block\]: (\d+)")):
            m = re.search(pat, block)
            f[key] = int(m.group(1)) if m else None
        figures[name] = f
    assert figures, "no resource report"
    return figures


def _one(usage, kernel, args):
    """The entry of kernel<args> (mangled names: k_photon<float> is k_photonIfE...)."""
    hits = [v for k, v in usage.items() if re.search(r"\d%s%sE" % (kernel, re.escape(args)), k)]
    assert len(hits) == 1, (kernel, args, [k for k in usage if kernel in k])
    return hits[0]


def test_photon_pass_keeps_four_waves(usage):
    f = _one(usage, "k_photon", "IfE")
    assert f["occ"] >= 4 and f["vgpr"] <= 128 and f["scratch"] == 0
    assert 4 * f["lds"] <= 160 * 1024


def test_lepton_passes(usage):
    assert _one(usage, "k_lepton", "IfLb0E")["occ"] >= 3
    assert _one(usage, "k_heavy", "IfLb0E")["occ"] >= 3
    assert _one(usage, "k_light", "IfLb0E")["occ"] >= 3
    assert _one(usage, "k_synchrotron", "IfLb1E")["occ"] == 8


def test_no_scratch(usage):
    """No kernel spills registers to scratch memory."""
    spill = sorted(k for k, f in usage.items() if f["scratch"])
    assert not spill, spill


def test_optical_depth_heavy_queue(usage):
    """Two 256-thread blocks per compute unit: the launch bound the kernel is compiled
    for, and what its LDS allows."""
    f = _one(usage, "k_heavy", "IfLb1E")
    assert f["occ"] >= 2 and f["scratch"] == 0
    assert 2 * f["lds"] <= 160 * 1024 < 3 * f["lds"]
