"""FP64 reference of the learned activation proposal's network (test
infrastructure: only tests, smoke and the benchmark's CPU leg use it).

A 12-64-64-1 perceptron: standardised input x' = (x - mean) * inv_std,
h1 = relu(W1 x' + b1), h2 = relu(W2 h1 + b2), z = w3 . h2 + b3, p = sigmoid(z);
loss = mean binary cross-entropy of z against labels y; Adam update as in
Kingma and Ba (2015), Algorithm 1, with bias-corrected moments.  Parameters
are one vector: mean[12], inv_std[12], W1[64][12], b1[64], W2[64][64], b2[64],
w3[64], b3[1].  Written from those definitions with numpy, no blocking.
"""
from __future__ import annotations

import numpy as np

IN, HID = 12, 64
SIZES = [("mean", (IN,)), ("inv_std", (IN,)), ("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)),
         ("b2", (HID,)), ("w3", (HID,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)
TRAINABLE_FROM = 2 * IN


def unpack(p: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def init_params(seed: int, mean=None, inv_std=None) -> np.ndarray:
    """He-uniform weights, zero biases (seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = {
        "mean": np.zeros(IN) if mean is None else mean,
        "inv_std": np.ones(IN) if inv_std is None else inv_std,
        "W1": rng.uniform(-1, 1, (HID, IN)) * np.sqrt(6.0 / IN),
        "b1": np.zeros(HID),
        "W2": rng.uniform(-1, 1, (HID, HID)) * np.sqrt(6.0 / HID),
        "b2": np.zeros(HID),
        "w3": rng.uniform(-1, 1, HID) * np.sqrt(6.0 / HID),
        "b3": np.zeros(1),
    }
    return pack(d)


def forward(p: np.ndarray, x: np.ndarray):
    """Logits and hidden activations for samples x [n, 12]."""
    d = unpack(p)
    xn = (np.asarray(x, np.float64) - d["mean"]) * d["inv_std"]
    h1 = np.maximum(xn @ d["W1"].T + d["b1"], 0.0)
    h2 = np.maximum(h1 @ d["W2"].T + d["b2"], 0.0)
    z = h2 @ d["w3"] + d["b3"][0]
    return z, h1, h2


def loss(p: np.ndarray, x: np.ndarray, y: np.ndarray) -> float:
    z, _, _ = forward(p, x)
    y = np.asarray(y, np.float64)
    # -[y log s(z) + (1 - y) log(1 - s(z))], written stably
    return float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def grad(p: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Gradient of loss() with respect to every parameter (the
    standardisation constants get 0: they are not trained)."""
    d = unpack(p)
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = x.shape[0]
    xn = (x - d["mean"]) * d["inv_std"]
    z, h1, h2 = forward(p, x)
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n          # d loss / d z
    dh2 = np.outer(dz, d["w3"]) * (h2 > 0)
    dh1 = (dh2 @ d["W2"]) * (h1 > 0)
    g = {
        "mean": np.zeros(IN), "inv_std": np.zeros(IN),
        "W1": dh1.T @ xn, "b1": dh1.sum(axis=0),
        "W2": dh2.T @ h1, "b2": dh2.sum(axis=0),
        "w3": h2.T @ dz, "b3": np.array([dz.sum()]),
    }
    return pack(g)


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on the trainable parameters; returns new (p, m, v)."""
    p, g, m, v = (np.array(a, np.float64) for a in (p, g, m, v))
    sl = slice(TRAINABLE_FROM, None)
    m[sl] = b1 * m[sl] + (1 - b1) * g[sl]
    v[sl] = b2 * v[sl] + (1 - b2) * g[sl] ** 2
    mh = m[sl] / (1 - b1 ** t)
    vh = v[sl] / (1 - b2 ** t)
    p[sl] = p[sl] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
