"""Exact K-nearest-neighbour search by definition -- oracle (test infrastructure).

Section 2.1 (KNNS problem): given n D-dimensional vectors and a query q,
return the k vectors minimising the squared Euclidean distance
delta(v, q) = sum_i (v_i - q_i)^2, the sum taken over the D coordinates
i = 0 .. D-1 (the printed upper bound "D" is read as D-1: there are D
coordinates).  The paper fixes no order among equal distances; results
here are ordered by (delta, row id) ascending.  When k exceeds the number
of rows the tail is padded with id -1 and distance +inf.

Every float32 input is widened exactly to float64 before any arithmetic.

The kernel listing of Section 3 gives two more distances over the same
layout: L1, sum_i |v_i - q_i|, and the inner product sum_i v_i q_i, whose
nearest neighbours are the largest values; here the inner product is
scored as its negation so that every metric ranks ascending.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libknn_fp64.so")


def sqdist(x: np.ndarray, q: np.ndarray) -> np.ndarray:
    """delta(v, q) for every row v of x, in float64 (Section 2.1)."""
    diff = np.asarray(x, dtype=np.float64) - np.asarray(q, dtype=np.float64)[None, :]
    return np.einsum("ij,ij->i", diff, diff)


def l1dist(x: np.ndarray, q: np.ndarray) -> np.ndarray:
    """sum_i |v_i - q_i| for every row v of x, in float64."""
    diff = np.asarray(x, dtype=np.float64) - np.asarray(q, dtype=np.float64)[None, :]
    return np.abs(diff).sum(axis=1)


def neg_ip(x: np.ndarray, q: np.ndarray) -> np.ndarray:
    """-sum_i v_i q_i for every row v of x, in float64."""
    return -(np.asarray(x, dtype=np.float64) @ np.asarray(q, dtype=np.float64))


METRICS = {"l2": sqdist, "l1": l1dist, "ip": neg_ip}


def topk_by_dist_then_id(dist: np.ndarray, ids: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
    """The k smallest (dist, id) pairs, ascending; pads with (-1, +inf)."""
    order = np.lexsort((ids, dist))[:k]
    out_i = np.full(k, -1, dtype=np.int64)
    out_d = np.full(k, np.inf, dtype=np.float64)
    out_i[: order.size] = ids[order]
    out_d[: order.size] = dist[order]
    return out_i, out_d


def knn_exact(x: np.ndarray, queries: np.ndarray, k: int, metric: str = "l2") -> Tuple[np.ndarray, np.ndarray]:
    """Brute-force exact KNN over the horizontal (row-major) layout, for the
    metric "l2" (the default), "l1" or "ip" (scored as -q.v).

    Returns (ids [nq, k] int64, dist [nq, k] float64).
    """
    score = METRICS[metric]
    x = np.asarray(x)
    queries = np.atleast_2d(np.asarray(queries))
    n = x.shape[0]
    ids = np.arange(n, dtype=np.int64)
    out_i = np.empty((queries.shape[0], k), dtype=np.int64)
    out_d = np.empty((queries.shape[0], k), dtype=np.float64)
    for qi in range(queries.shape[0]):
        out_i[qi], out_d[qi] = topk_by_dist_then_id(score(x, queries[qi]), ids, k)
    return out_i, out_d


def knn_exact_blocked(x: np.ndarray, queries: np.ndarray, k: int, metric: str = "l2",
                      block: int = 65536) -> Tuple[np.ndarray, np.ndarray]:
    """:func:`knn_exact` over blocks of rows (every query against one block
    at a time, keeping each query's k best so far), for collections too
    large to widen to float64 at once.  Same results."""
    x = np.asarray(x)
    queries = np.atleast_2d(np.asarray(queries, dtype=np.float64))
    nq = queries.shape[0]
    best_i = np.full((nq, 0), -1, dtype=np.int64)
    best_d = np.zeros((nq, 0), dtype=np.float64)
    for b0 in range(0, x.shape[0], block):
        xb = np.asarray(x[b0:b0 + block], dtype=np.float64)
        ids = np.arange(b0, b0 + xb.shape[0], dtype=np.int64)
        if metric == "ip":
            sc = -(queries @ xb.T)
        elif metric == "l1":
            sc = np.stack([np.abs(xb - qq[None, :]).sum(1) for qq in queries])
        else:
            sc = np.stack([((xb - qq[None, :]) ** 2).sum(1) for qq in queries])
        new_i = np.empty((nq, min(k, best_i.shape[1] + ids.size)), dtype=np.int64)
        new_d = np.empty(new_i.shape, dtype=np.float64)
        for qi in range(nq):
            di = np.concatenate([best_d[qi], sc[qi]])
            ii = np.concatenate([best_i[qi], ids])
            o = np.lexsort((ii, di))[: new_i.shape[1]]
            new_i[qi], new_d[qi] = ii[o], di[o]
        best_i, best_d = new_i, new_d
    out_i = np.full((nq, k), -1, dtype=np.int64)
    out_d = np.full((nq, k), np.inf, dtype=np.float64)
    out_i[:, : best_i.shape[1]] = best_i
    out_d[:, : best_d.shape[1]] = best_d
    return out_i, out_d


# --------------------------------------------------------------------------
# The same definition in plain C (double accumulation, one coordinate at a
# time), for the large inputs the numpy version is too slow for.
# --------------------------------------------------------------------------

_lib: Optional[ctypes.CDLL] = None


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle C library not built: {_LIB_PATH} (run oracle/build.py)")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_knn_fp64.restype = ctypes.c_int
        lib.oracle_knn_fp64.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
        ]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def c_threads() -> int:
    """Threads the C oracle's OpenMP runtime will use."""
    return int(_load().oracle_max_threads())


def knn_exact_c(x: np.ndarray, queries: np.ndarray, k: int,
                threads: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Exact KNN through the plain C implementation (same definition and tie
    order as :func:`knn_exact`).  ``threads=0`` uses every available core."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    queries = np.ascontiguousarray(np.atleast_2d(queries), dtype=np.float32)
    n, d = x.shape
    nq = queries.shape[0]
    if queries.shape[1] != d:
        raise ValueError("dimension mismatch")
    out_i = np.empty((nq, k), dtype=np.int64)
    out_d = np.empty((nq, k), dtype=np.float64)
    rc = lib.oracle_knn_fp64(x.ctypes.data, n, d, queries.ctypes.data, nq, k,
                             out_i.ctypes.data, out_d.ctypes.data, threads)
    if rc != 0:
        raise RuntimeError(f"oracle_knn_fp64 failed with code {rc}")
    return out_i, out_d


def recall_at_k(truth_ids: np.ndarray, got_ids: np.ndarray) -> float:
    """Mean over queries of |R intersect R_hat| / k (Section 2.1)."""
    truth_ids = np.atleast_2d(truth_ids)
    got_ids = np.atleast_2d(got_ids)
    k = truth_ids.shape[1]
    hits = 0
    for t, g in zip(truth_ids, got_ids):
        hits += len(set(int(v) for v in t if v >= 0) & set(int(v) for v in g if v >= 0))
    return hits / (k * truth_ids.shape[0])
