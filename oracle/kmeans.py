"""Lloyd k-means for the IVF buckets, and index invariants -- oracle
(test infrastructure).

Section 2.1 (IVF): the collection is grouped into buckets by a
non-optimised Lloyd algorithm; a vector belongs to the bucket of its
nearest centroid.  The paper gives no initialisation, iteration count or
empty-cluster rule.  Readings used here: the initial centroids are the
rows whose indices the caller passes in (drawn from a seed), a fixed
number of iterations is run, every iteration first assigns each row to
its nearest centroid (equal distances: lower centroid id) and then moves
every non-empty centroid to the mean of its members; an empty bucket
keeps its previous centroid.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def assign(x: np.ndarray, centroids: np.ndarray, block: int = 4096) -> Tuple[np.ndarray, np.ndarray]:
    """Nearest centroid per row (ties: lower id) and its squared distance."""
    x = np.asarray(x, dtype=np.float64)
    c = np.asarray(centroids, dtype=np.float64)
    lab = np.empty(x.shape[0], dtype=np.int64)
    dist = np.empty(x.shape[0], dtype=np.float64)
    for s in range(0, x.shape[0], block):
        xb = x[s:s + block]
        diff = xb[:, None, :] - c[None, :, :]
        dd = np.einsum("ijk,ijk->ij", diff, diff)
        lab[s:s + block] = np.argmin(dd, axis=1)  # first minimum = lowest id
        dist[s:s + block] = dd[np.arange(xb.shape[0]), lab[s:s + block]]
    return lab, dist


def update(x: np.ndarray, lab: np.ndarray, prev: np.ndarray) -> np.ndarray:
    """Mean of each bucket's members; empty buckets keep ``prev``."""
    x = np.asarray(x, dtype=np.float64)
    k = prev.shape[0]
    sums = np.zeros((k, x.shape[1]))
    np.add.at(sums, lab, x)
    cnt = np.bincount(lab, minlength=k)
    out = np.array(prev, dtype=np.float64, copy=True)
    nz = cnt > 0
    out[nz] = sums[nz] / cnt[nz, None]
    return out


def lloyd(x: np.ndarray, init_rows: np.ndarray, iters: int) -> Tuple[np.ndarray, np.ndarray, List[float]]:
    """Returns (centroids [k, D] float64, labels [n], objective per step).

    The objective list holds the within-bucket sum of squares after each
    assignment step (iters + 1 values: one per update plus the final
    assignment)."""
    x = np.asarray(x, dtype=np.float64)
    c = x[np.asarray(init_rows, dtype=np.int64)].copy()
    obj = []
    for _ in range(iters):
        lab, dist = assign(x, c)
        obj.append(float(dist.sum()))
        c = update(x, lab, c)
    lab, dist = assign(x, c)
    obj.append(float(dist.sum()))
    return c, lab, obj


def lists_from_labels(lab: np.ndarray, k: int) -> List[np.ndarray]:
    """Bucket member ids, ascending within each bucket."""
    lab = np.asarray(lab, dtype=np.int64)
    order = np.argsort(lab, kind="stable")
    bounds = np.searchsorted(lab[order], np.arange(k + 1))
    return [order[bounds[i]:bounds[i + 1]] for i in range(k)]


def check_nearest(x: np.ndarray, centroids: np.ndarray, lab: np.ndarray, rel: float = 1e-5) -> int:
    """Number of rows whose bucket centroid is farther than the nearest one
    by more than ``rel`` relative (0 for a valid final assignment)."""
    _, best = assign(x, centroids)
    c = np.asarray(centroids, dtype=np.float64)
    diff = np.asarray(x, dtype=np.float64) - c[np.asarray(lab, dtype=np.int64)]
    got = np.einsum("ij,ij->i", diff, diff)
    return int(np.sum(got > best * (1.0 + rel) + 1e-30))
