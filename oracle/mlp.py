"""The learned early-termination network, forward and backward in float64 --
oracle (test infrastructure).

The paper prunes with fixed rules; this network is an addition beside the
ADSampling test (a learned stop decision per query and probe checkpoint).
Architecture: x (F = 72 inputs) -> h1 = relu(W1 x + b1) (64)
-> h2 = relu(W2 h1 + b2) (64) -> z = w3 . h2 + b3, p = sigmoid(z) is the
probability that stopping here loses nothing.  The search uses the weights
rounded to float16, so the oracle evaluates the same rounded weights.

Loss (mean over n samples, y in {0, 1}, negatives weighted by w0 because a
wrong stop costs recall):
    L = (1/n) sum( -y log p - w0 (1 - y) log(1 - p) ),  dL/dz = (1/n)(-y (1-p) + w0 (1-y) p).

Parameter vector layout (float32 on the device, float64 here):
W1 [64][72] | b1 [64] | W2 [64][64] | b2 [64] | w3 [64] | b3 [1], padded to 8960.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

F_IN = 72
H = 64
SIZES = [("W1", (H, F_IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
P_USED = sum(int(np.prod(s)) for _, s in SIZES)
P_PAD = 8960


def unpack(theta: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    return out


def pack(parts: Dict[str, np.ndarray]) -> np.ndarray:
    theta = np.zeros(P_PAD, dtype=np.float64)
    o = 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        theta[o:o + size] = np.asarray(parts[name], dtype=np.float64).ravel()
        o += size
    return theta


def fp16_round(theta: np.ndarray) -> np.ndarray:
    return np.asarray(theta, dtype=np.float32).astype(np.float16).astype(np.float64)


def forward(theta: np.ndarray, x: np.ndarray) -> Tuple[np.ndarray, Dict[str, np.ndarray]]:
    p = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["w3"] + p["b3"][0]
    return z, {"x": x, "a1": a1, "h1": h1, "a2": a2, "h2": h2}


def sigmoid(z: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-z))


def loss(theta: np.ndarray, x: np.ndarray, y: np.ndarray, w0: float) -> float:
    z, _ = forward(theta, x)
    y = np.asarray(y, dtype=np.float64)
    # log p = -softplus(-z), log(1-p) = -softplus(z)
    sp_neg = np.logaddexp(0.0, -z)
    sp_pos = np.logaddexp(0.0, z)
    return float(np.mean(y * sp_neg + w0 * (1.0 - y) * sp_pos))


def grad(theta: np.ndarray, x: np.ndarray, y: np.ndarray, w0: float) -> np.ndarray:
    """Analytic gradient of :func:`loss` (backpropagation by the chain rule)."""
    z, c = forward(theta, x)
    p = unpack(theta)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    s = sigmoid(z)
    dz = (-y * (1.0 - s) + w0 * (1.0 - y) * s) / n
    g = {"w3": c["h2"].T @ dz, "b3": np.array([dz.sum()])}
    dh2 = np.outer(dz, p["w3"]) * (c["a2"] > 0)
    g["W2"] = dh2.T @ c["h1"]
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ p["W2"]) * (c["a1"] > 0)
    g["W1"] = dh1.T @ c["x"]
    g["b1"] = dh1.sum(0)
    return pack(g)


def numeric_grad(theta: np.ndarray, x: np.ndarray, y: np.ndarray, w0: float, idx, h: float = 1e-6) -> np.ndarray:
    """Central finite differences of :func:`loss` at the given parameter indices."""
    out = np.empty(len(idx))
    for t, i in enumerate(idx):
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        out[t] = (loss(tp, x, y, w0) - loss(tm, x, y, w0)) / (2 * h)
    return out
