"""CPU oracle of the cost-model MLP (test infrastructure only).

The MLP maps 4 leaf features to a predicted join time: x -> ReLU(W1 x + b1)
-> ReLU(W2 h1 + b2) -> w3 . h2 + b3.  Parameters are used after rounding to
BF16 (round to nearest, ties to even, of their binary32 values); everything
else is float64 here.  Loss L = mean_s (y_s - t_s)^2.  Adam (Kingma & Ba,
"Adam: A method for stochastic optimization", ICLR 2015) with the usual
bias correction updates FP32 master parameters.

Parameter vector layout (4545 values): W1[64][4], b1[64], W2[64][64],
b2[64], w3[64], b3.  This module shares no code with the HIP kernels.
"""
from __future__ import annotations

import numpy as np

H, F = 64, 4
SIZES = [("W1", H * F), ("b1", H), ("W2", H * H), ("b2", H), ("w3", H), ("b3", 1)]
P = sum(n for _, n in SIZES)


def bf16_bits(x) -> np.ndarray:
    """BF16 bit patterns (uint16) of binary32 values, round to nearest even."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    r = np.where(nan, ((u >> 16) | 0x40) & 0xFFFF, r)
    return r.astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    return (np.asarray(bits, np.uint32) << 16).view(np.float32)


def bf16_round(x) -> np.ndarray:
    return bf16_value(bf16_bits(x))


def unpack(p):
    p = np.asarray(p, np.float64)
    out, o = {}, 0
    for name, n in SIZES:
        out[name] = p[o:o + n]
        o += n
    out["W1"] = out["W1"].reshape(H, F)
    out["W2"] = out["W2"].reshape(H, H)
    out["b3"] = out["b3"][0]
    return out


def forward(p, X):
    """Predictions for samples X [n, 4]; p are the (already rounded)
    parameters."""
    q = unpack(p)
    X = np.asarray(X, np.float64)
    h1 = np.maximum(X @ q["W1"].T + q["b1"], 0.0)
    h2 = np.maximum(h1 @ q["W2"].T + q["b2"], 0.0)
    return h2 @ q["w3"] + q["b3"]


def loss_grad(p, X, T):
    """(L, dL/dp) for L = mean (y - t)^2, by backpropagation in float64."""
    q = unpack(p)
    X = np.asarray(X, np.float64)
    T = np.asarray(T, np.float64)
    n = len(T)
    a1 = X @ q["W1"].T + q["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ q["w3"] + q["b3"]
    r = y - T
    L = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    d2 = np.outer(dy, q["w3"]) * (a2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ q["W2"]) * (a1 > 0)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(axis=0)
    return L, np.concatenate([g[name].ravel() for name, _ in SIZES])


def adam_step(master, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in float64; returns (master, m, v)."""
    master, grad, m, v = (np.asarray(a, np.float64) for a in (master, grad, m, v))
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return master - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initialisation (float32 masters)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(P, np.float32)
    o = 0
    for name, n in SIZES:
        if name == "W1":
            p[o:o + n] = rng.normal(0, np.sqrt(2.0 / F), n)
        elif name == "W2":
            p[o:o + n] = rng.normal(0, np.sqrt(2.0 / H), n)
        elif name == "w3":
            p[o:o + n] = rng.normal(0, np.sqrt(1.0 / H), n)
        o += n
    return p
