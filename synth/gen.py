"""Seeded Gaussian-mixture generators shaped like the paper's workloads.

The paper evaluates on public embedding collections (Section 2.2, the
"Vector Datasets" table: GIST/960, OpenAI/1536, Contriever and arXiv/768,
...).  None of them is available here, so every input is drawn from a
seeded mixture whose shape and value distribution stand in for them:

* ``isotropic``   -- normal-looking data (DEEP/SIFT-like), small config.
* ``skewed``      -- per-dimension spreads decaying from 1 to ~0.18 in a
                     random dimension order (GIST-like "skewed" class of
                     Section 2.2), the exact-search workload.
* ``anisotropic`` -- unit-norm rows from an uneven mixture with random
                     per-component scales (LLM-embedding-like, OpenAI /
                     Contriever), the IVF workloads.

Determinism: every stream (component parameters, database rows, query
rows) comes from its own ``numpy.random.SeedSequence`` child, and rows are
drawn in fixed blocks with per-block children, so any slice of rows can
be regenerated on its own and the result never depends on how many rows
were requested together.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

_BLOCK = 4096  # rows per independently seeded block (always drawn whole)

_STREAM_PARAMS = 0
_STREAM_DATA = 1
_STREAM_QUERY = 2


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(entropy=seed, spawn_key=tuple(key)))


@dataclass
class Mixture:
    """A finite Gaussian mixture with diagonal per-component spreads."""

    means: np.ndarray            # [C, D] float32
    scales: np.ndarray           # [C, D] float32 standard deviations
    weights: np.ndarray          # [C] float64, sums to 1
    seed: int
    normalize: bool = False
    info: Dict[str, object] = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return int(self.means.shape[1])

    def _block(self, stream: int, qseed: int, b: int) -> np.ndarray:
        rows = _BLOCK
        lab = _rng(self.seed, stream, qseed, b, 0).choice(self.weights.shape[0], size=rows, p=self.weights)
        z = _rng(self.seed, stream, qseed, b, 1).standard_normal((rows, self.dim), dtype=np.float32)
        x = self.means[lab] + self.scales[lab] * z
        if self.normalize:
            nrm = np.sqrt(np.einsum("ij,ij->i", x, x, dtype=np.float64)).astype(np.float32)
            nrm[nrm == 0] = 1.0
            x /= nrm[:, None]
        return x

    def rows(self, n: int, stream: int = _STREAM_DATA, qseed: int = 0,
             start: int = 0) -> np.ndarray:
        """Rows ``start .. start+n-1`` of a stream, as float32 [n, D]."""
        out = np.empty((n, self.dim), dtype=np.float32)
        pieces = []  # (block, offset in block, rows, position in out)
        pos = 0
        r = start
        while pos < n:
            b, off = divmod(r, _BLOCK)
            take = min(_BLOCK - off, n - pos)
            pieces.append((b, off, take, pos))
            pos += take
            r += take

        def fill(piece):
            b, off, take, at = piece
            out[at:at + take] = self._block(stream, qseed, b)[off:off + take]

        if len(pieces) > 2:
            workers = min(16, os.cpu_count() or 1, len(pieces))
            with ThreadPoolExecutor(workers) as ex:
                list(ex.map(fill, pieces))
        else:
            for pc in pieces:
                fill(pc)
        return out

    def data(self, n: int, start: int = 0) -> np.ndarray:
        return self.rows(n, _STREAM_DATA, 0, start)

    def labels(self, n: int, start: int = 0) -> np.ndarray:
        """Mixture component of data rows ``start .. start+n-1`` (int32)."""
        out = np.empty(n, dtype=np.int32)
        pos, r = 0, start
        while pos < n:
            b, off = divmod(r, _BLOCK)
            take = min(_BLOCK - off, n - pos)
            lab = _rng(self.seed, _STREAM_DATA, 0, b, 0).choice(self.weights.shape[0], size=_BLOCK, p=self.weights)
            out[pos:pos + take] = lab[off:off + take]
            pos += take
            r += take
        return out

    def queries(self, nq: int, query_seed: Optional[int] = None) -> np.ndarray:
        qs = self.seed if query_seed is None else query_seed
        return self.rows(nq, _STREAM_QUERY, qs, 0)


def isotropic_mixture(d: int = 128, components: int = 16, mean_var: float = 4.0,
                      seed: int = 42) -> Mixture:
    """Uniform weights; means ~ N(0, mean_var I); unit-variance noise."""
    rng = _rng(seed, _STREAM_PARAMS)
    means = (np.sqrt(mean_var) * rng.standard_normal((components, d))).astype(np.float32)
    scales = np.ones((components, d), dtype=np.float32)
    w = np.full(components, 1.0 / components)
    return Mixture(means, scales, w, seed, False, {"kind": "isotropic"})


def skewed_mixture(d: int = 960, components: int = 64, decay: float = 32.0,
                   mean_var: float = 4.0, seed: int = 42) -> Mixture:
    """Per-dimension spread sigma_{perm(j)} = 1/sqrt(1 + j/decay) over a random
    dimension permutation; means ~ N(0, mean_var diag(sigma^2))."""
    rng = _rng(seed, _STREAM_PARAMS)
    perm = rng.permutation(d)
    sig = np.empty(d, dtype=np.float64)
    sig[perm] = 1.0 / np.sqrt(1.0 + np.arange(d) / decay)
    means = (np.sqrt(mean_var) * sig[None, :] * rng.standard_normal((components, d))).astype(np.float32)
    scales = np.broadcast_to(sig.astype(np.float32), (components, d)).copy()
    w = np.full(components, 1.0 / components)
    return Mixture(means, scales, w, seed, False, {"kind": "skewed", "sigma": sig})


def anisotropic_unit_mixture(d: int = 1536, components: int = 256, seed: int = 42) -> Mixture:
    """Dirichlet(1) weights (uneven clusters); means ~ N(0, I); per-component
    per-dimension spreads 0.5*exp(0.5*zeta), zeta ~ N(0,1); rows scaled to
    unit L2 norm."""
    rng = _rng(seed, _STREAM_PARAMS)
    w = rng.dirichlet(np.ones(components))
    means = rng.standard_normal((components, d)).astype(np.float32)
    scales = (0.5 * np.exp(0.5 * rng.standard_normal((components, d)))).astype(np.float32)
    return Mixture(means, scales, w, seed, True, {"kind": "anisotropic"})


def integer_grid(n: int, d: int, nq: int, lo: int = -8, hi: int = 8,
                 seed: int = 7) -> Tuple[np.ndarray, np.ndarray]:
    """Integer-valued float32 data and queries, uniform on {lo..hi}^d.

    With d <= 2048 every partial and full squared distance is an integer
    below 2**24, hence exact in float32 and float64 alike.
    """
    rng = _rng(seed, 99)
    x = rng.integers(lo, hi + 1, size=(n, d)).astype(np.float32)
    q = rng.integers(lo, hi + 1, size=(nq, d)).astype(np.float32)
    return x, q


def standard_normal(n: int, d: int, nq: int, seed: int = 11) -> Tuple[np.ndarray, np.ndarray]:
    """The kernel study's collections (Section 6.4): n vectors and nq
    queries of d independent N(0, 1) float32 values."""
    rng = _rng(seed, 101, d)
    x = rng.standard_normal((n, d), dtype=np.float32)
    q = rng.standard_normal((nq, d), dtype=np.float32)
    return x, q


# the kernel study's grid (Section 6.4): collection sizes 64 .. 131,072 and
# these dimensionalities
KERNEL_STUDY_N = (64, 1024, 16384, 131072)
KERNEL_STUDY_D = (8, 16, 32, 64, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 4096, 8192)
KERNEL_STUDY_BLOCKS = (16, 32, 64, 128, 256, 512)


# name -> (mixture factory, full n, full nq, query seed)
WORKLOADS = {
    # exact linear scan: 10,000 x 128, 100 queries
    "linear_10k_d128": (lambda: isotropic_mixture(128, 16, 4.0, 42), 10_000, 100, None),
    # exact PDX-BOND: 1,000,000 x 960 skewed, 1,000 queries
    "bond_1m_d960": (lambda: skewed_mixture(960, 64, 32.0, 4.0, 42), 1_000_000, 1_000, None),
    # IVF + ADSampling: 1,000,000 x 1536 unit-norm, 10,000 queries
    "ivf_1m_d1536": (lambda: anisotropic_unit_mixture(1536, 256, 42), 1_000_000, 10_000, None),
    # low precision: 5,000,000 x 768 unit-norm, 10,000 queries
    "lowp_5m_d768": (lambda: anisotropic_unit_mixture(768, 256, 42), 5_000_000, 10_000, None),
    # learned pruning, GIST-like IVF: training queries seed 43, evaluation 44
    "mlp_train_1m_d960": (lambda: skewed_mixture(960, 64, 32.0, 4.0, 42), 1_000_000, 10_000, 43),
    "mlp_eval_1m_d960": (lambda: skewed_mixture(960, 64, 32.0, 4.0, 42), 1_000_000, 10_000, 44),
}


def workload(name: str, n: Optional[int] = None, nq: Optional[int] = None):
    """Return (X [n, D] float32, Q [nq, D] float32, Mixture) for a named workload,
    optionally truncated to the first n rows / nq queries."""
    fac, n_full, nq_full, qseed = WORKLOADS[name]
    mix = fac()
    n = n_full if n is None else n
    nq = nq_full if nq is None else nq
    return mix.data(n), mix.queries(nq, qseed), mix
