"""Pins of the FP64 network reference used to check the GPU training kernels:
finite differences of the loss, the activation's closed forms and the
bfloat16 rounding rule."""
import numpy as np

from oracle import mlp_ref


def _setup(seed=0, n=96):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.3, mlp_ref.NPARAMS)
    smp = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(0, 2, n),
                    rng.uniform(0.1, 2.0, n)], axis=1)
    return p, smp


def test_gradient_matches_finite_differences():
    p, smp = _setup()
    L, g = mlp_ref.gradient(p, smp)
    assert abs(L - mlp_ref.loss(p, smp)) <= 1e-15 * max(1.0, L)
    rng = np.random.default_rng(1)
    # a few parameters of every tensor
    idx = []
    for name, off in mlp_ref.OFF.items():
        size = {"W1": 128, "b1": 64, "W2": 4096, "b2": 64, "W3": 4096, "b3": 64, "W4": 64, "b4": 1}[name]
        idx += list(off + rng.choice(size, min(size, 6), replace=False))
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (mlp_ref.loss(pp, smp) - mlp_ref.loss(pm, smp)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_activation_closed_forms():
    t = np.linspace(-50, 50, 2001)
    a = mlp_ref.act(t)
    assert np.all(np.abs(a) < 1) and np.all(np.diff(a) > 0)
    assert np.allclose(mlp_ref.act(-t), -a)
    # derivative against a central difference
    h = 1e-5
    fd = (mlp_ref.act(t + h) - mlp_ref.act(t - h)) / (2 * h)
    assert np.allclose(fd, mlp_ref.dact(t), rtol=1e-7, atol=1e-10)
    assert abs(mlp_ref.act(np.array([1e8]))[0] - 1.0) < 1e-15


def test_bf16_rounding_rule():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -8 + 2 ** -20, -2.5, 3.0e38])
    r = mlp_ref.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # halfway: to even
    assert r[2] == 1.0 + 2 ** -6           # halfway: to even (upwards)
    assert r[3] == 1.0 + 2 ** -7           # above halfway
    assert r[4] == -2.5
    assert abs(r[5] / 3.0e38 - 1) < 2 ** -8


def test_pack_unpack_roundtrip():
    p, _ = _setup(3)
    assert np.array_equal(mlp_ref.pack(mlp_ref.unpack(p)), p)
