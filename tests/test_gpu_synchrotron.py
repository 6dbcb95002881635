"""GPU parity of qed_synchrotron against the oracle's F, G (Sec. 3.2.1)."""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2008_10468_amd import qed
    cfg = qed.qed_config_default()
    cfg.stream = torch.cuda.current_stream().cuda_stream
    c = qed.qed_init(cfg)
    yield c
    qed.qed_finalize(c)


def _points():
    grid = 10.0 ** np.linspace(-7, math.log10(700.0), 4001)
    rand = workloads.c4_host(20000, seed=5)
    # segment boundaries of both tables in t = x^(1/3), +-2 ulp
    edges = np.concatenate([(0.5 * np.arange(1, 10)) ** 3, (0.25 * np.arange(1, 38)) ** 3])
    bnd = np.concatenate([np.nextafter(np.nextafter(edges, 0), 0), np.nextafter(edges, 0), edges,
                          np.nextafter(edges, np.inf), np.nextafter(np.nextafter(edges, np.inf), np.inf)])
    return np.concatenate([grid, rand, bnd])


@pytest.mark.parametrize("dtype,tol,xmax", [("float32", 2e-6, 80.0), ("float64", 1e-12, 700.0)])
def test_synchrotron_matches_oracle(ctx, dtype, tol, xmax):
    from paper_2008_10468_amd import qed
    x = _points()
    x = x[x <= xmax]
    td = getattr(torch, dtype)
    xg = torch.from_numpy(x).to(td).cuda()
    F, G = qed.synchrotron(ctx, xg)
    st, rep = qed.qed_sync(ctx)
    assert st == qed.QED_OK
    xe = xg.double().cpu().numpy()          # the exact inputs the kernel saw
    Fo, Go = oracle.synchrotron_parallel(xe)
    eF = np.abs(F.double().cpu().numpy() / Fo - 1)
    eG = np.abs(G.double().cpu().numpy() / Go - 1)
    print(f"{dtype}: max rel err F {eF.max():.3e} G {eG.max():.3e}")
    assert eF.max() <= tol and eG.max() <= tol


@pytest.mark.parametrize("n", [1, 255, 257, 100003])
def test_ragged_sizes_and_null_outputs(ctx, n):
    from paper_2008_10468_amd import qed
    x = torch.from_numpy(workloads.c4_host(n, seed=n)).float().cuda()
    F = torch.full_like(x, -1.0)
    assert qed.qed_synchrotron(ctx, x.data_ptr(), F.data_ptr(), None, n, qed.QED_F32) == qed.QED_OK
    assert qed.qed_sync(ctx)[0] == qed.QED_OK
    Fo, _ = oracle.synchrotron(x.double().cpu().numpy())
    assert np.max(np.abs(F.double().cpu().numpy() / Fo - 1)) <= 2e-6


@pytest.mark.parametrize("dtype,tol", [("float32", 2e-6), ("float64", 1e-12)])
@pytest.mark.parametrize("n", [1, 3, 1001, 65537])
def test_unaligned_pointers_and_tails(ctx, dtype, tol, n):
    """Arrays that start one element past a 16-byte boundary take the one-element-per-lane
    kernel; aligned arrays of a length that is not a whole number of vectors take the
    vector kernel and its tail.  Both against the oracle, in float and double."""
    from paper_2008_10468_amd import qed
    td = getattr(torch, dtype)
    code = qed.QED_F32 if dtype == "float32" else qed.QED_F64
    xs = workloads.c4_host(n, seed=n + 7)
    Fo, Go = oracle.synchrotron(np.asarray(torch.from_numpy(xs).to(td).double().numpy()))
    for off in (0, 1):
        x = torch.zeros(n + 1, dtype=td, device="cuda")
        x[off:off + n] = torch.from_numpy(xs).to(td).cuda()
        F = torch.full((n + 1,), -1.0, dtype=td, device="cuda")
        G = torch.full((n + 1,), -1.0, dtype=td, device="cuda")
        es = x.element_size() * off
        assert ((x.data_ptr() + es) % 16 != 0) == (off == 1)
        assert qed.qed_synchrotron(ctx, x.data_ptr() + es, F.data_ptr() + es, G.data_ptr() + es, n, code) == qed.QED_OK
        assert qed.qed_sync(ctx)[0] == qed.QED_OK
        f = F.double().cpu().numpy()
        g = G.double().cpu().numpy()
        assert np.max(np.abs(f[off:off + n] / Fo - 1)) <= tol and np.max(np.abs(g[off:off + n] / Go - 1)) <= tol
        rest = np.concatenate([f[:off], f[off + n:]])
        assert np.all(rest == -1.0)                     # nothing written outside the n outputs


def test_edge_values(ctx):
    from paper_2008_10468_amd import qed
    for td in (torch.float32, torch.float64):
        x = torch.tensor([0.0, float("inf"), 1e4, -1.0, float("nan")], dtype=td).cuda()
        F, G = qed.synchrotron(ctx, x)
        st, rep = qed.qed_sync(ctx)
        assert st == qed.QED_ERR_NONFINITE and rep.nonfinite == 2
        f = F.cpu().numpy()
        g = G.cpu().numpy()
        assert f[0] == 0 and g[0] == 0 and f[1] == 0 and g[1] == 0 and f[2] == 0
        assert np.isnan(f[3]) and np.isnan(g[4])
    # status cleared after sync
    assert qed.qed_sync(ctx)[0] == qed.QED_OK


def test_invalid_arguments(ctx):
    from paper_2008_10468_amd import qed
    x = torch.ones(4, device="cuda")
    assert qed.qed_synchrotron(ctx, x.data_ptr(), None, None, 4, qed.QED_F32) == qed.QED_ERR_INVALID_ARG
    assert qed.qed_synchrotron(ctx, x.data_ptr(), x.data_ptr(), None, 4, 7) == qed.QED_ERR_INVALID_ARG
    assert qed.qed_synchrotron(ctx, None, x.data_ptr(), None, 4, qed.QED_F32) == qed.QED_ERR_INVALID_ARG
    assert qed.qed_synchrotron(ctx, None, None, None, 0, qed.QED_F32) == qed.QED_OK
