"""The PDX layout by definition -- oracle (test infrastructure).

Section 3 and its kernel listing: vectors are cut into vectorgroups of G
(64 in the paper) and, inside a group, all values of one dimension are
stored next to each other, so dimension d of the group's n-th vector
sits at offset d*G + n.  Here the last group is padded with zeros up to G
vectors (the paper is silent on a ragged tail).

Per-dimension collection means (the "distance to means" statistics of
Section 5) are computed in float64 and rounded once to float32, the
precision of the stored vectors.
"""
from __future__ import annotations

import numpy as np


def to_pdx(x: np.ndarray, group: int = 64) -> np.ndarray:
    """[n, D] row-major -> [ceil(n/G), D, G] (zero-padded last group)."""
    x = np.asarray(x, dtype=np.float32)
    n, d = x.shape
    ng = (n + group - 1) // group
    out = np.zeros((ng, d, group), dtype=np.float32)
    for v in range(n):
        g, lane = divmod(v, group)
        out[g, :, lane] = x[v]
    return out


def from_pdx(p: np.ndarray, n: int) -> np.ndarray:
    """Inverse of :func:`to_pdx` (drops the padding lanes)."""
    ng, d, group = p.shape
    out = np.empty((n, d), dtype=p.dtype)
    for v in range(n):
        g, lane = divmod(v, group)
        out[v] = p[g, :, lane]
    return out


def column_means(x: np.ndarray) -> np.ndarray:
    """Per-dimension mean over all rows, accumulated in float64."""
    return np.asarray(x, dtype=np.float64).mean(axis=0)


def column_means_f32(x: np.ndarray) -> np.ndarray:
    """The stored form of the means: float64 mean rounded once to float32."""
    return column_means(x).astype(np.float32)
