"""PDXearch, PDX-BOND, ADSampling and IVF-flat, step by step -- oracle
(test infrastructure).

What is followed, in the paper's order:

* Section 4 (PDXearch framework): the search walks blocks one after the
  other.  START: the first block is scanned without pruning to obtain a
  threshold (here: blocks keep being scanned fully until k candidates
  exist; before that the threshold is +inf).  Every later block is
  scanned dimension-chunk by dimension-chunk; after each chunk a pruning
  predicate is evaluated on the partial distances.  WARMUP keeps computing
  all vectors of the block; once the share of not-yet-pruned vectors falls
  below a selection threshold (20 %, Section 6.1 "Parameters"), PRUNE
  computes only the survivors.  After the last dimension the survivors are
  merged into the k-best list and the threshold becomes its k-th distance.
  WARMUP vs PRUNE changes only which values are computed, never the result.
* Section 2.3 (exact bounds) and Section 5 (PDX-BOND): the bound is the
  partial distance itself; a vector is pruned when it is strictly higher
  than the threshold (the current k-th best exact distance).  Dimensions
  are visited in decreasing order of |q_j - mean_j| (distance to means),
  or (dimension zones) zone by zone, zones ranked by that criterion.
* Section 2.3 (ADSampling): on randomly rotated vectors, visited in their
  natural order, every delta_d dimensions the partial distance is tested
  against the threshold with the error bound eps0.  The paper describes
  the test in words only; the formula is the one of the cited ADSampling
  method: after d of D dimensions the estimate partial*D/d is compared
  with tau*(1 + eps0/sqrt(d))^2, and at d = D the comparison is exact.
  Parameters (Section 6.1): delta_d = 32 (D/4 when D < 128), eps0 = 2.1.
* Section 2.3 (BSA): a PCA projection of the collection, and a test by
  error quantiles from the Cauchy-Schwarz inequality with a multiplier m
  instead of the hypothesis test.  The paper states it in words only; the
  reading used here: after d dimensions the unseen part of the distance,
  |q_r|^2 + |x_r|^2 - 2 q_r.x_r over the remaining dimensions, is estimated
  by replacing q_r.x_r with m |q_r| |x_r| (the Cauchy-Schwarz maximum when
  m = 1, which makes the estimate a lower bound and the search exact within
  the probed buckets), and a vector is dropped when partial + max(that, 0)
  exceeds the threshold; at d = D the comparison is exact.
* Section 2.1 (IVF): distances to all centroids first, then the vectors in
  the nprobe nearest buckets; buckets are visited nearest first (ties by
  bucket id) and the first one is the START block.

All arithmetic is float64; float32 inputs are widened exactly.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from .exact import sqdist, topk_by_dist_then_id


# --------------------------------------------------------------------------
# dimension orders and chunking
# --------------------------------------------------------------------------

def bond_order(q: np.ndarray, mu32: np.ndarray) -> np.ndarray:
    """PDX-BOND visit order (Section 5, distance to means): dimensions by
    |q_j - mean_j| descending, equal keys by j ascending.  The key is formed
    in float32, the precision of the stored vectors and means."""
    key = np.abs(np.asarray(q, dtype=np.float32) - np.asarray(mu32, dtype=np.float32))
    return np.argsort(-key, kind="stable").astype(np.int64)


def zone_order(q: np.ndarray, mu32: np.ndarray, zone: int = 32) -> np.ndarray:
    """Dimension zones (Section 5, Figure "dz"): runs of `zone` consecutive
    stored dimensions, ranked by the summed distance to means
    sum_j |q_j - mean_j| of their dimensions, most promising first; inside a
    zone the dimensions keep their storage order.  Readings (the paper fixes
    neither): equal scores go by zone index ascending, and when D is not a
    multiple of `zone` the shorter last zone is visited last, so that every
    fetch of `zone` dimensions is one whole zone.  zone = 1 is the
    distance-to-means order, zone = D the natural order."""
    key = np.abs(np.asarray(q, dtype=np.float32) - np.asarray(mu32, dtype=np.float32)).astype(np.float64)
    d = key.size
    nz = d // zone
    score = key[: nz * zone].reshape(nz, zone).sum(axis=1)
    rank = np.argsort(-score, kind="stable")
    full = (rank[:, None] * zone + np.arange(zone)[None, :]).reshape(-1)
    return np.concatenate([full, np.arange(nz * zone, d)]).astype(np.int64)


def ads_delta_d(d: int) -> int:
    """Section 6.1: delta_d = 32, or D/4 when D < 128."""
    return 32 if d >= 128 else max(1, d // 4)


def fixed_chunks(order: np.ndarray, chunk: int) -> List[np.ndarray]:
    return [order[i:i + chunk] for i in range(0, order.size, chunk)]


def doubling_chunks(order: np.ndarray, first: int = 2) -> List[np.ndarray]:
    """Section 4 WARMUP: fetch 2, then 4, then 8, ... dimensions."""
    out, i, step = [], 0, first
    while i < order.size:
        out.append(order[i:i + step])
        i += step
        step *= 2
    return out


# --------------------------------------------------------------------------
# pruning predicates: prune(partial, tau, dims_seen, D) -> bool array
# --------------------------------------------------------------------------

def bond_prunes(partial: np.ndarray, tau: float, dims_seen: int, d: int) -> np.ndarray:
    """Exact bound: the partial distance is a lower bound (Section 2.3)."""
    return partial > tau


def make_ads_prunes(eps0: float) -> Callable[[np.ndarray, float, int, int], np.ndarray]:
    """ADSampling hypothesis test with error bound eps0 (Section 2.3)."""

    def prune(partial: np.ndarray, tau: float, dims_seen: int, d: int) -> np.ndarray:
        if dims_seen >= d or not np.isfinite(eps0):
            return partial > tau
        ratio = d / dims_seen
        bound = tau * (1.0 + eps0 / np.sqrt(dims_seen)) ** 2
        return partial * ratio > bound

    return prune


def make_bsa_prunes(xb: np.ndarray, qv: np.ndarray, m: float) -> Callable[[np.ndarray, float, int, int], np.ndarray]:
    """BSA's test (Section 2.3, reading above) for the rows xb of one block
    and the query qv (both in the rotated space, visited in natural order):
    drop iff partial + max(|q_r|^2 + |x_r|^2 - 2 m |q_r| |x_r|, 0) > tau
    with r the dimensions not yet seen; exact at d = D."""
    xb = np.asarray(xb, dtype=np.float64)
    qv = np.asarray(qv, dtype=np.float64)

    def prune(partial: np.ndarray, tau: float, dims_seen: int, d: int) -> np.ndarray:
        if dims_seen >= d:
            return partial > tau
        xr = np.sqrt((xb[:, dims_seen:] ** 2).sum(axis=1))
        qr = float(np.sqrt((qv[dims_seen:] ** 2).sum()))
        rest = np.maximum(qr * qr + xr * xr - 2.0 * m * qr * xr, 0.0)
        return partial + rest > tau

    return prune


def bsa_ivf_search(xrot: np.ndarray, lists: Sequence[np.ndarray], centroids: np.ndarray,
                   qrot: np.ndarray, k: int, nprobe: int, m: float, delta_d: Optional[int] = None,
                   switch: float = 0.2, stats: Optional[SearchStats] = None) -> Tuple[np.ndarray, np.ndarray]:
    """PDXearch with BSA's test inside IVF (Sections 2.3, 4): probed buckets
    nearest first, dimensions in natural (rotated) order, tests every
    delta_d dimensions."""
    xrot = np.asarray(xrot)
    d = xrot.shape[1]
    dd = ads_delta_d(d) if delta_d is None else delta_d
    probe = ivf_probe_order(centroids, qrot, nprobe)
    blocks = [np.asarray(lists[p], dtype=np.int64) for p in probe]
    prunes = [make_bsa_prunes(xrot[b], qrot, m) for b in blocks]
    return pdxearch(xrot, qrot, k, blocks, fixed_chunks(np.arange(d), dd), prunes, switch, stats)


def never_prunes(partial: np.ndarray, tau: float, dims_seen: int, d: int) -> np.ndarray:
    return np.zeros(partial.shape, dtype=bool)


# --------------------------------------------------------------------------
# PDXearch
# --------------------------------------------------------------------------

@dataclass
class SearchStats:
    values_computed: int = 0      # (vector, dimension) values evaluated
    values_total: int = 0         # values a linear scan of the same blocks would evaluate
    survivors_per_chunk: List[int] = field(default_factory=list)

    @property
    def pruning_power(self) -> float:
        """Share of dimension values not used (Section 2.3, pruning power)."""
        return 1.0 - self.values_computed / max(1, self.values_total)


class _KBest:
    def __init__(self, k: int):
        self.k = k
        self.d = np.empty(0, dtype=np.float64)
        self.i = np.empty(0, dtype=np.int64)

    def merge(self, dist: np.ndarray, ids: np.ndarray) -> None:
        d = np.concatenate([self.d, dist])
        i = np.concatenate([self.i, ids])
        o = np.lexsort((i, d))[: self.k]
        self.d, self.i = d[o], i[o]

    @property
    def tau(self) -> float:
        return float(self.d[-1]) if self.d.size == self.k else np.inf

    def result(self) -> Tuple[np.ndarray, np.ndarray]:
        return topk_by_dist_then_id(self.d, self.i, self.k)


def pdxearch(x: np.ndarray, q: np.ndarray, k: int, blocks: Sequence[np.ndarray],
             chunks: Sequence[np.ndarray], prune: Callable, switch: float = 0.2,
             stats: Optional[SearchStats] = None) -> Tuple[np.ndarray, np.ndarray]:
    """PDXearch over ``blocks`` (arrays of row ids) with a fixed dimension
    chunking ``chunks`` (arrays of dimension indices covering 0..D-1 once).
    ``prune`` is one predicate for every block, or a sequence with one per
    block.

    Returns (ids [k], dist [k]) ordered by (dist, id); pads with (-1, inf).
    """
    x = np.asarray(x)
    qq = np.asarray(q, dtype=np.float64)
    d = x.shape[1]
    best = _KBest(k)
    st = stats if stats is not None else SearchStats()
    prunes = list(prune) if isinstance(prune, (list, tuple)) else [prune] * len(blocks)
    for rows, prune_b in zip(blocks, prunes):
        rows = np.asarray(rows, dtype=np.int64)
        if rows.size == 0:
            continue
        st.values_total += rows.size * d
        xb = np.asarray(x[rows], dtype=np.float64)
        if best.tau == np.inf:
            # START: linear scan, no threshold yet
            best.merge(sqdist(xb, qq), rows)
            st.values_computed += rows.size * d
            continue
        tau = best.tau
        partial = np.zeros(rows.size, dtype=np.float64)
        alive = np.ones(rows.size, dtype=bool)
        warmup = True
        seen = 0
        for ch in chunks:
            comp = np.ones(rows.size, dtype=bool) if warmup else alive.copy()
            diff = xb[np.ix_(comp, ch)] - qq[ch][None, :]
            partial[comp] += np.einsum("ij,ij->i", diff, diff)
            st.values_computed += int(comp.sum()) * ch.size
            seen += ch.size
            alive &= ~prune_b(partial, tau, seen, d)
            st.survivors_per_chunk.append(int(alive.sum()))
            if warmup and alive.mean() < switch:
                warmup = False
            if not alive.any():
                break
        if alive.any():
            surv = rows[alive]
            # survivors carry their complete distance; report it by definition
            best.merge(sqdist(x[surv], qq), surv)
    return best.result()


def bond_search(x: np.ndarray, q: np.ndarray, k: int, block: int = 10_000, chunk: int = 32,
                mu32: Optional[np.ndarray] = None, switch: float = 0.2,
                stats: Optional[SearchStats] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Exact PDX-BOND search (Sections 4, 5, 6.5): horizontal blocks of at
    most ``block`` rows, distance-to-means order, fixed chunks."""
    x = np.asarray(x)
    n, d = x.shape
    if mu32 is None:
        mu32 = np.asarray(x, dtype=np.float64).mean(axis=0).astype(np.float32)
    order = bond_order(q, mu32)
    blocks = [np.arange(s, min(n, s + block)) for s in range(0, n, block)]
    return pdxearch(x, q, k, blocks, fixed_chunks(order, chunk), bond_prunes, switch, stats)


def bond_search_batch(x: np.ndarray, queries: np.ndarray, k: int, **kw):
    queries = np.atleast_2d(queries)
    out = [bond_search(x, q, k, **kw) for q in queries]
    return np.stack([o[0] for o in out]), np.stack([o[1] for o in out])


# --------------------------------------------------------------------------
# IVF
# --------------------------------------------------------------------------

def ivf_probe_order(centroids: np.ndarray, qrot: np.ndarray, nprobe: int) -> np.ndarray:
    """The nprobe buckets with the smallest centroid distance, nearest
    first, equal distances by bucket id (Section 2.1, IVF)."""
    dist = sqdist(centroids, qrot)
    return np.lexsort((np.arange(dist.size), dist))[:nprobe].astype(np.int64)


def ivf_flat(xrot: np.ndarray, lists: Sequence[np.ndarray], centroids: np.ndarray,
             qrot: np.ndarray, k: int, nprobe: int) -> Tuple[np.ndarray, np.ndarray]:
    """Exact top-k over the union of the probed buckets (IVF_FLAT)."""
    probe = ivf_probe_order(centroids, qrot, nprobe)
    rows = np.concatenate([np.asarray(lists[p], dtype=np.int64) for p in probe]) if probe.size else np.empty(0, np.int64)
    if rows.size == 0:
        return topk_by_dist_then_id(np.empty(0), np.empty(0, np.int64), k)
    return topk_by_dist_then_id(sqdist(np.asarray(xrot)[rows], qrot), rows, k)


def ads_ivf_search(xrot: np.ndarray, lists: Sequence[np.ndarray], centroids: np.ndarray,
                   qrot: np.ndarray, k: int, nprobe: int, eps0: float = 2.1,
                   delta_d: Optional[int] = None, switch: float = 0.2,
                   stats: Optional[SearchStats] = None) -> Tuple[np.ndarray, np.ndarray]:
    """PDXearch with the ADSampling test inside IVF (Sections 2.3, 4, 6.2):
    probed buckets nearest first, rotated dimensions in natural order,
    checkpoints every delta_d dimensions."""
    xrot = np.asarray(xrot)
    d = xrot.shape[1]
    dd = ads_delta_d(d) if delta_d is None else delta_d
    probe = ivf_probe_order(centroids, qrot, nprobe)
    blocks = [np.asarray(lists[p], dtype=np.int64) for p in probe]
    return pdxearch(xrot, qrot, k, blocks, fixed_chunks(np.arange(d), dd),
                    make_ads_prunes(eps0), switch, stats)


def bond_ivf_search(xrot: np.ndarray, lists: Sequence[np.ndarray], centroids: np.ndarray,
                    qrot: np.ndarray, k: int, nprobe: int, mu32: np.ndarray, chunk: int = 32,
                    zone: Optional[int] = None, switch: float = 0.2,
                    stats: Optional[SearchStats] = None) -> Tuple[np.ndarray, np.ndarray]:
    """PDX-BOND inside IVF (Section 5 within Section 2.1's IVF): the probed
    buckets nearest first (the first is START), dimensions in the query's
    distance-to-means order (zone None) or in dimension zones of `zone`
    dimensions, fetched `chunk` at a time, a vector dropped once its partial
    distance exceeds the k-th best.  mu32: per-dimension means of the stored
    rows.  Exact within the probed buckets."""
    xrot = np.asarray(xrot)
    probe = ivf_probe_order(centroids, qrot, nprobe)
    blocks = [np.asarray(lists[p], dtype=np.int64) for p in probe]
    order = bond_order(qrot, mu32) if zone is None else zone_order(qrot, mu32, zone)
    return pdxearch(xrot, qrot, k, blocks, fixed_chunks(order, chunk), bond_prunes, switch, stats)


def make_table_prunes(mult_row: np.ndarray, delta_d: int) -> Callable[[np.ndarray, float, int, int], np.ndarray]:
    """The ADSampling-shaped test with a multiplier per test point in place
    of (1 + eps0/sqrt(d))^2: after dims_seen = (c + 1) delta_d < D
    dimensions, drop iff partial * D/dims_seen > tau * mult_row[c]; exact
    after all D dimensions."""

    def prune(partial: np.ndarray, tau: float, dims_seen: int, d: int) -> np.ndarray:
        if dims_seen >= d:
            return partial > tau
        return partial * (d / dims_seen) > tau * mult_row[dims_seen // delta_d - 1]

    return prune


def learned_ivf_search(xrot: np.ndarray, lists: Sequence[np.ndarray], centroids: np.ndarray,
                       qrot: np.ndarray, k: int, nprobe: int, mult: np.ndarray, delta_d: int,
                       switch: float = 0.2, stats: Optional[SearchStats] = None) -> Tuple[np.ndarray, np.ndarray]:
    """:func:`ads_ivf_search` with the learned multipliers mult [nprobe-1][C]
    (row r - 1 for the bucket of probe rank r; the START bucket, rank 0, is
    scanned whole)."""
    xrot = np.asarray(xrot)
    d = xrot.shape[1]
    probe = ivf_probe_order(centroids, qrot, nprobe)
    blocks = [np.asarray(lists[p], dtype=np.int64) for p in probe]
    prunes = [never_prunes] + [make_table_prunes(mult[r - 1], delta_d) for r in range(1, len(blocks))]
    return pdxearch(xrot, qrot, k, blocks, fixed_chunks(np.arange(d), delta_d), prunes, switch, stats)
