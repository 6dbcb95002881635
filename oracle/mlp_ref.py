"""FP64 reference of the surrogate sampler's network (test infrastructure only).

Used by the tests to check the GPU training kernels' loss and gradients; nothing
in the library imports it.  The network maps (s, v) to y through three hidden
layers of 64 units with activation a(t) = t / sqrt(1 + t^2):

    h1 = a(W1 [s, v] + b1),  h2 = a(W2 h1 + b2),  h3 = a(W3 h2 + b3),  y = W4 h3 + b4,

and the training loss of a batch of n rows (s, v, y_t, w) is
(1/n) sum w (y - y_t)^2.  Parameters are one flat vector in the order W1[64][2],
b1, W2[64][64], b2, W3[64][64], b3, W4[64], b4 (weights stored [out][in]).

`round_bf16` optionally rounds the two 64 x 64 layers' weights the way the
GPU's matrix cores see them: each weight as the sum of two bfloat16 numbers
(hi = bf16(w), lo = bf16(w - hi), round to nearest even), so a check can separate
that rounding from the rest (the activations, also held as hi + lo on the GPU,
are kept exact here).  This module's own correctness is
pinned by finite differences of `loss` (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np

H = 64
NPARAMS = 8577
OFF = {"W1": 0, "b1": 128, "W2": 192, "b2": 4288, "W3": 4352, "b3": 8448, "W4": 8512, "b4": 8576}


def unpack(p):
    p = np.asarray(p, np.float64)
    return {
        "W1": p[0:128].reshape(H, 2), "b1": p[128:192],
        "W2": p[192:4288].reshape(H, H), "b2": p[4288:4352],
        "W3": p[4352:8448].reshape(H, H), "b3": p[8448:8512],
        "W4": p[8512:8576], "b4": p[8576],
    }


def pack(d):
    return np.concatenate([d["W1"].ravel(), d["b1"], d["W2"].ravel(), d["b2"], d["W3"].ravel(), d["b3"],
                           d["W4"], np.atleast_1d(d["b4"])])


def bf16(x):
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def split_bf16(x):
    """x as the sum of two bfloat16 numbers: bf16(x) + bf16(x - bf16(x))."""
    hi = bf16(x)
    return hi + bf16(np.asarray(x, np.float64) - hi)


def act(t):
    return t / np.sqrt(1.0 + t * t)


def dact(t):
    return (1.0 + t * t) ** -1.5


def forward(p, s, v, round_bf16=False):
    d = unpack(p)
    x = np.stack([s, v], axis=1).astype(np.float64)
    z1 = x @ d["W1"].T + d["b1"]
    h1 = act(z1)
    W2, W3 = (split_bf16(d["W2"]), split_bf16(d["W3"])) if round_bf16 else (d["W2"], d["W3"])
    z2 = h1 @ W2.T + d["b2"]
    h2 = act(z2)
    z3 = h2 @ W3.T + d["b3"]
    h3 = act(z3)
    y = h3 @ d["W4"] + d["b4"]
    return y, (x, z1, h1, z2, h2, z3, h3)


def loss(p, samples, round_bf16=False):
    s, v, yt, w = (samples[:, k].astype(np.float64) for k in range(4))
    y, _ = forward(p, s, v, round_bf16)
    return float(np.mean(w * (y - yt) ** 2))


def gradient(p, samples, round_bf16=False):
    """(loss, d loss / d p) by backpropagation."""
    s, v, yt, w = (samples[:, k].astype(np.float64) for k in range(4))
    n = s.size
    d = unpack(p)
    y, (x, z1, h1, z2, h2, z3, h3) = forward(p, s, v, round_bf16)
    W2, W3 = (split_bf16(d["W2"]), split_bf16(d["W3"])) if round_bf16 else (d["W2"], d["W3"])
    e = y - yt
    L = float(np.mean(w * e * e))
    dy = 2.0 * w * e / n
    g = {"b4": np.sum(dy), "W4": h3.T @ dy}
    dz3 = np.outer(dy, d["W4"]) * dact(z3)
    g["b3"] = dz3.sum(0)
    g["W3"] = dz3.T @ h2
    dz2 = (dz3 @ W3) * dact(z2)
    g["b2"] = dz2.sum(0)
    g["W2"] = dz2.T @ h1
    dz1 = (dz2 @ W2) * dact(z1)
    g["b1"] = dz1.sum(0)
    g["W1"] = dz1.T @ x
    return L, pack(g)
