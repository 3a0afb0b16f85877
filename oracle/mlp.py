"""Oracle: the per-vertex warm-start MLP in FP64 numpy (test infrastructure).

Same architecture and parameter layout as the GPU kernels:
9 (padded to 16) -> 128 -> 128 -> 128 -> 3 (padded to 16), SiLU activations,
mean-squared error over the first n_out outputs, Adam with bias correction.
Forward and backward are written out layer by layer (plain matrix products).
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 16, 128, 16
SHAPES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (HID, OUT)), ("b4", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([d[name].ravel() for name, _ in SHAPES])


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init(seed=0, n_in=9, n_out=3):
    """He-style init; padded input rows and output columns are zero."""
    rng = np.random.default_rng(seed)
    d = {}
    d["W1"] = np.zeros((IN, HID))
    d["W1"][:n_in] = rng.normal(size=(n_in, HID)) * np.sqrt(2.0 / n_in)
    d["b1"] = np.zeros(HID)
    d["W2"] = rng.normal(size=(HID, HID)) * np.sqrt(2.0 / HID)
    d["b2"] = np.zeros(HID)
    d["W3"] = rng.normal(size=(HID, HID)) * np.sqrt(2.0 / HID)
    d["b3"] = np.zeros(HID)
    d["W4"] = np.zeros((HID, OUT))
    d["W4"][:, :n_out] = rng.normal(size=(HID, n_out)) * np.sqrt(1.0 / HID)
    d["b4"] = np.zeros(OUT)
    return pack(d)


def forward(p, x):
    w = unpack(p)
    Z1 = x @ w["W1"] + w["b1"]
    H1 = silu(Z1)
    Z2 = H1 @ w["W2"] + w["b2"]
    H2 = silu(Z2)
    Z3 = H2 @ w["W3"] + w["b3"]
    H3 = silu(Z3)
    y = H3 @ w["W4"] + w["b4"]
    return y, (Z1, H1, Z2, H2, Z3, H3)


def mse(y, t, n_out=3):
    d = np.zeros_like(y)
    d[:, :n_out] = y[:, :n_out] - t[:, :n_out]
    B = y.shape[0]
    return float(np.sum(d * d) / (B * n_out)), 2.0 * d / (B * n_out)


def backward(p, x, act, dy):
    w = unpack(p)
    Z1, H1, Z2, H2, Z3, H3 = act
    g = {}
    g["W4"] = H3.T @ dy
    g["b4"] = dy.sum(0)
    dZ3 = (dy @ w["W4"].T) * silu_grad(Z3)
    g["W3"] = H2.T @ dZ3
    g["b3"] = dZ3.sum(0)
    dZ2 = (dZ3 @ w["W3"].T) * silu_grad(Z2)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2 @ w["W2"].T) * silu_grad(Z1)
    g["W1"] = x.T @ dZ1
    g["b1"] = dZ1.sum(0)
    return pack(g)


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
