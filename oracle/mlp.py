"""The search's learned networks, forward and backward in float64 --
oracle (test infrastructure).

The paper prunes with fixed rules; these networks are additions beside the
ADSampling test (Section 2.3) and the fixed-nprobe IVF search (Section
2.1): a per-query probe budget (a stop decision per probe count) and a
per-(query, bucket) error bound for the ADSampling-shaped prune test.
Architecture: x (F = 72 inputs) -> h1 = relu(W1 x + b1) (64)
-> h2 = relu(W2 h1 + b2) (64) -> z = w3 . h2 + b3.  The search uses the
weights rounded to float16, so the oracle evaluates the same rounded
weights.

Losses (mean over n samples):
* "bce", stop decision, y in {0, 1}, p = sigmoid(z) the probability that
  stopping loses nothing, negatives weighted by w0 because a wrong stop
  costs recall:
      L = (1/n) sum( -y log p - w0 (1 - y) log(1 - p) ),
      dL/dz = (1/n)(-y (1-p) + w0 (1-y) p);
* "pinball" at level w in (0, 1), prune bound, y a real target, z
  then estimates the w-quantile of y (quantile regression):
      L = (1/n) sum( u (w - [u < 0]) ),  u = y - z,
      dL/dz = (1/n)([z > y] - w).

Prune bound: the network gives each (query, bucket of probe rank r >= 1)
an error bound eps = scale * z; after c1 of D dimensions the multiplier
m = max(1 + eps/sqrt(c1), 0)^2 (capped at 1e30) replaces ADSampling's
(1 + eps0/sqrt(c1))^2 in the test partial * D/c1 > tau * m.

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


def loss(theta: np.ndarray, x: np.ndarray, y: np.ndarray, w0: float, kind: str = "bce") -> float:
    z, _ = forward(theta, x)
    y = np.asarray(y, dtype=np.float64)
    if kind == "pinball":
        u = y - z
        return float(np.mean(u * (w0 - (u < 0))))
    # log p = -softplus(-z), log(1-p) = -softplus(z)
    sp_neg = np.logaddexp(0.0, -z)
    sp_pos = np.logaddexp(0.0, z)
    return float(np.mean(y * sp_neg + w0 * (1.0 - y) * sp_pos))


def dloss_dz(z: np.ndarray, y: np.ndarray, w0: float, kind: str = "bce") -> np.ndarray:
    """Per-sample derivative of :func:`loss` with respect to z (already divided by n)."""
    n = z.shape[0]
    if kind == "pinball":
        return ((z > y).astype(np.float64) - w0) / n
    s = sigmoid(z)
    return (-y * (1.0 - s) + w0 * (1.0 - y) * s) / n


def grad(theta: np.ndarray, x: np.ndarray, y: np.ndarray, w0: float, kind: str = "bce") -> np.ndarray:
    """Analytic gradient of :func:`loss` (backpropagation by the chain rule)."""
    z, c = forward(theta, x)
    p = unpack(theta)
    y = np.asarray(y, dtype=np.float64)
    dz = dloss_dz(z, y, w0, kind)
    g = {"w3": c["h2"].T @ dz, "b3": np.array([dz.sum()])}
    dh2 = np.outer(dz, p["w3"]) * (c["a2"] > 0)
    g["W2"] = dh2.T @ c["h1"]
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ p["W2"]) * (c["a1"] > 0)
    g["W1"] = dh1.T @ c["x"]
    g["b1"] = dh1.sum(0)
    return pack(g)


def numeric_grad(theta: np.ndarray, x: np.ndarray, y: np.ndarray, w0: float, idx, h: float = 1e-6,
                 kind: str = "bce") -> np.ndarray:
    """Central finite differences of :func:`loss` at the given parameter indices."""
    out = np.empty(len(idx))
    for t, i in enumerate(idx):
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        out[t] = (loss(tp, x, y, w0, kind) - loss(tm, x, y, w0, kind)) / (2 * h)
    return out


# --------------------------------------------------------------------------
# prune bound: inputs, multipliers, training targets
# --------------------------------------------------------------------------

def prune_inputs(qrot: np.ndarray, tau: float, cd: np.ndarray, r: int, nprobe: int) -> np.ndarray:
    """The 72 inputs for the bucket of probe rank r >= 1: the first 64
    rotated query coordinates (zero-padded), then tau/d_r, d_r/d_0, tau/d_0
    (each clamped to [0, 1e4]) and log2(r)/log2(nprobe), then 4 zeros.
    tau: the k-th distance in the START bucket; cd: squared centroid
    distances of the probed buckets, nearest first."""
    d = qrot.shape[0]
    x = np.zeros(F_IN, dtype=np.float64)
    m = min(d, 64)
    x[:m] = qrot[:m]
    d0, dr = max(cd[0], 1e-20), max(cd[r], 1e-20)  # a zero distance is read as 1e-20
    x[64:67] = np.clip(np.array([tau / dr, dr / d0, tau / d0], dtype=np.float64), 0.0, 1e4)
    x[67] = np.log2(r) / np.log2(nprobe)
    return x


def test_points(d: int, delta_d: int):
    """The dimension counts c1 = delta_d, 2 delta_d, ... below D after which
    the prune test runs (the test after all D dimensions is exact)."""
    return list(range(delta_d, d, delta_d))


def multiplier(eps: float, c1: int) -> float:
    """max(1 + eps/sqrt(c1), 0)^2, capped at 1e30."""
    b = max(1.0 + eps / np.sqrt(c1), 0.0)
    return min(b * b, 1e30)


def prune_multipliers(theta: np.ndarray, qrot: np.ndarray, tau: float, cd: np.ndarray, nprobe: int,
                      delta_d: int, scale: float = 1.0) -> np.ndarray:
    """m [nprobe - 1][C] of one query: row r - 1 for probe rank r."""
    pts = test_points(qrot.shape[0], delta_d)
    if nprobe < 2:
        return np.zeros((0, len(pts)))
    z, _ = forward(theta, np.stack([prune_inputs(qrot, tau, cd, r, nprobe) for r in range(1, nprobe)]))
    return np.array([[multiplier(scale * e, c1) for c1 in pts] for e in z])


def prune_targets(xrot: np.ndarray, qrot: np.ndarray, ids: np.ndarray, tau_k: float, delta_d: int) -> np.ndarray:
    """[len(ids)]: the smallest eps keeping each id at every test point,
    max over c1 of (sqrt(partial(c1) D / (c1 tau_k)) - 1) sqrt(c1), with
    partial(c1) the squared distance over the first c1 rotated dimensions."""
    d = qrot.shape[0]
    diff = np.asarray(xrot, dtype=np.float64)[np.asarray(ids, dtype=np.int64)] - qrot[None, :]
    pref = np.cumsum(diff * diff, axis=1)
    out = np.full(len(ids), -np.inf)
    for c1 in test_points(d, delta_d):
        out = np.maximum(out, (np.sqrt(pref[:, c1 - 1] * d / (c1 * tau_k)) - 1.0) * np.sqrt(c1))
    return out
