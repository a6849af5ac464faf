"""Low-precision vector storage -- oracle (test infrastructure).

The paper keeps float32 vectors and names compressed PDX blocks as future
work (Section 7, "PDX storage designs").  The storage forms checked here are
the ones the search library offers beside float32, written from the formats'
definitions:

* bfloat16: the upper 16 bits of the float32 pattern after rounding to
  nearest, ties to even.
* float8 e4m3 ("fn" variant, OCP 8-bit floating point): 1 sign bit, 4
  exponent bits (bias 7), 3 mantissa bits; no infinities; largest finite
  magnitude 448; subnormals m * 2^-9.  Encoding rounds to nearest, ties to
  even, and saturates at +-448.  Every dimension j has a scale
  s_j = max_i |x_ij| / 448 (float32 division; 1 when the column is all
  zero) and the stored code is e4m3(x_ij / s_j).

Distances over the decoded values are the plain definition of Section 2.1.
"""
from __future__ import annotations

import numpy as np


# ----------------------------- bfloat16 ------------------------------------

def bf16_encode(x: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    return ((b + 0x7FFF + lsb) >> 16).astype(np.uint16)


def bf16_decode(code: np.ndarray) -> np.ndarray:
    return (np.asarray(code, dtype=np.uint32) << 16).view(np.float32)


# ----------------------------- float8 e4m3 ---------------------------------

E4M3_MAX = 448.0


def fp8_scales(x: np.ndarray) -> np.ndarray:
    m = np.abs(np.asarray(x, dtype=np.float32)).max(axis=0)
    s = (m / np.float32(E4M3_MAX)).astype(np.float32)
    s[m == 0] = 1.0
    return s


def _e4m3_encode_scalar(v: float) -> int:
    """Round-to-nearest-even encoding of one float32 value (saturating)."""
    sign = 0x80 if np.signbit(np.float32(v)) else 0
    a = abs(float(np.float32(v)))
    if a == 0.0:
        return sign
    if a >= E4M3_MAX:
        return sign | 0x7E
    e = int(np.floor(np.log2(a)))
    # guard against log2 rounding at exact powers of two
    if 2.0 ** e > a:
        e -= 1
    if 2.0 ** (e + 1) <= a:
        e += 1
    if e < -6:
        q = int(np.rint(a * 512.0))          # subnormal: multiples of 2^-9, ties to even
        return sign | q                       # q = 8 is the smallest normal, code 0x08
    m = a / 2.0 ** e - 1.0                    # in [0, 1)
    q = int(np.rint(m * 8.0))                 # 3 mantissa bits, ties to even
    code = ((e + 7) << 3) + q                 # q = 8 carries into the exponent
    return sign | min(code, 0x7E)


def e4m3_encode(v: np.ndarray) -> np.ndarray:
    flat = np.asarray(v, dtype=np.float32).ravel()
    out = np.fromiter((_e4m3_encode_scalar(t) for t in flat), dtype=np.uint8, count=flat.size)
    return out.reshape(np.shape(v))


def e4m3_encode_array(v: np.ndarray) -> np.ndarray:
    """The same encoding as ``e4m3_encode``, step for step, over whole
    arrays (for large inputs; the two agree on every value tested)."""
    x = np.asarray(v, dtype=np.float32)
    sign = np.where(np.signbit(x), 0x80, 0).astype(np.int32)
    a = np.abs(x).astype(np.float64)
    code = np.zeros(x.shape, dtype=np.int32)
    big = a >= E4M3_MAX
    pos = (a > 0) & ~big
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(pos, a, 1.0))).astype(np.int64)
    e = np.where(2.0 ** e > a, e - 1, e)          # log2 rounding at exact powers of two
    e = np.where(2.0 ** (e + 1) <= a, e + 1, e)
    sub = pos & (e < -6)
    q_sub = np.rint(a * 512.0).astype(np.int32)    # multiples of 2^-9, ties to even
    m = a / 2.0 ** e - 1.0
    q = np.rint(m * 8.0).astype(np.int64)          # 3 mantissa bits, ties to even
    c_norm = np.minimum(((e + 7) << 3) + q, 0x7E).astype(np.int32)
    code = np.where(sub, q_sub, np.where(pos, c_norm, code))
    code = np.where(big, 0x7E, code)
    return (sign | code).astype(np.uint8)


def e4m3_decode(code: np.ndarray) -> np.ndarray:
    c = np.asarray(code, dtype=np.int32)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 7
    val = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * 2.0 ** (e - 7.0))
    return (sign * val).astype(np.float32)


def fp8_encode(x: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """Codes of x / s_j (float32 division) per dimension."""
    y = (np.asarray(x, dtype=np.float32) / np.asarray(scales, dtype=np.float32)[None, :]).astype(np.float32)
    return e4m3_encode(y)


def fp8_encode_array(x: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """``fp8_encode`` through ``e4m3_encode_array`` (large inputs)."""
    y = (np.asarray(x, dtype=np.float32) / np.asarray(scales, dtype=np.float32)[None, :]).astype(np.float32)
    return e4m3_encode_array(y)


def fp8_decode(code: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """Decoded value e4m3(code) * s_j, as the float32 product."""
    return (e4m3_decode(code) * np.asarray(scales, dtype=np.float32)[None, :]).astype(np.float32)


# ----------------------------- rerank --------------------------------------

def rerank(x_exact: np.ndarray, x_approx: np.ndarray, rows: np.ndarray, q: np.ndarray, k: int, r: int):
    """Top-r of ``rows`` by the approximate distance (ties by id), then the
    top-k of those by the exact distance.  Returns (ids, exact dists)."""
    from .exact import sqdist, topk_by_dist_then_id
    rows = np.asarray(rows, dtype=np.int64)
    ai, _ = topk_by_dist_then_id(sqdist(np.asarray(x_approx)[rows], q), rows, r)
    ai = ai[ai >= 0]
    return topk_by_dist_then_id(sqdist(np.asarray(x_exact)[ai], q), ai, k)
