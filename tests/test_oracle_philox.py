"""Pins of the oracle's counter-based generator and uniform conversions."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

# Known-answer vectors published with Random123 for philox4x32 with 10 rounds.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(orc, ctr, key, out):
    assert tuple(int(v) for v in orc.philox(ctr, key)[0]) == out


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  unsigned long long seed = strtoull(argv[1], 0, 0), sub = strtoull(argv[2], 0, 0);
  int n = atoi(argv[3]);
  rocrand_state_philox4x32_10 st;
  rocrand_init(seed, sub, 0, &st);
  for (int k = 0; k < n; ++k) { uint4 r = rocrand4(&st); printf("%u %u %u %u\n", r.x, r.y, r.z, r.w); }
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_engine(orc):
    """rocRAND's host-callable Philox4x32-10 engine, used as a library: the k-th
    block of subsequence s under seed K is Philox((k, 0, s_lo, s_hi), (K_lo, K_hi))."""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.cpp")
        exe = os.path.join(d, "p")
        open(src, "w").write(ROCRAND_PROBE)
        subprocess.check_call(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", src, "-o", exe])
        for seed, sub in ((0x0123456789ABCDEF, 5), (1, 0), (0xFFFFFFFF00000001, (1 << 33) + 7)):
            out = subprocess.check_output([exe, str(seed), str(sub), "64"], text=True)
            got = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], np.uint32)
            ctr = np.zeros((64, 4), np.uint32)
            ctr[:, 0] = np.arange(64)
            ctr[:, 2] = sub & 0xFFFFFFFF
            ctr[:, 3] = sub >> 32
            key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)
            assert np.array_equal(orc.philox(ctr, key), got)


def test_uniform_conversions_exact(orc):
    # endpoints of the 53-bit and 24-bit conversions, strictly inside (0, 1)
    assert orc.u53(0, 0) == 2.0 ** -53
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert orc.u24(0) == 2.0 ** -24
    assert orc.u24(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    # value = (2k+1) 2^-b with k the top bits
    assert orc.u53(0x80000000, 0) == 0.5 + 2.0 ** -53
    assert orc.u24(0x80000000) == 0.5 + 2.0 ** -24
    # 24-bit values are exactly representable in float32
    for w in (0, 1, 511, 512, 0x12345678, 0xFFFFFE00, 0xFFFFFFFF):
        v = orc.u24(w)
        assert float(np.float32(v)) == v


def test_draw_layout(orc):
    seed, pid, step = 0x1234_5678_9ABC_DEF0, 0xDEAD_BEEF_0000_0042, 17
    key = (seed & 0xFFFFFFFF, seed >> 32)
    # 53-bit mode: one block per sub-step
    w = orc.philox((pid & 0xFFFFFFFF, pid >> 32, step, 9), key)[0]
    assert orc.draw_xy(seed, pid, step, 9, 53) == (orc.u53(w[0], w[1]), orc.u53(w[2], w[3]))
    # 24-bit mode: one block per pair of sub-steps
    w = orc.philox((pid & 0xFFFFFFFF, pid >> 32, step, 4), key)[0]
    assert orc.draw_xy(seed, pid, step, 8, 24) == (orc.u24(w[0]), orc.u24(w[1]))
    assert orc.draw_xy(seed, pid, step, 9, 24) == (orc.u24(w[2]), orc.u24(w[3]))


def test_uniform_statistics(orc):
    n = 200000
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    w = orc.philox(ctr, (7, 9))
    x = (((w[:, 0].astype(np.uint64) << 32) | w[:, 1]) >> 12).astype(np.float64) * 2.0 ** -52
    h, _ = np.histogram(x, bins=50, range=(0, 1))
    chi2 = float(np.sum((h - n / 50) ** 2 / (n / 50)))
    assert chi2 < 100          # 49 dof; p ~ 1e-5
    assert abs(np.corrcoef(x[:-1], x[1:])[0, 1]) < 0.01


def test_child_ids_distinct(orc):
    ids = {orc.child_id(1, p, s, i, slot) for p in range(20) for s in range(3) for i in range(20)
           for slot in (0, 1)}
    assert len(ids) == 20 * 3 * 20 * 2
