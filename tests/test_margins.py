"""The rounding margin of the matrix-core L2 linear mode, checked on the CPU.

The linear mode lists a vector when d' - e is at or below a bound, where
d' = |q|^2 + |x|^2 - 2 q.x comes from float32 matrix products and
e = 4 (D + 64) 2^-24 (|q|^2 + |x|^2).  Exactness rests on d' - e <= d <= d' + e
for the float32 distance d that the exact paths report (a fixed-order
chunked sum of squared differences).  This emulates both sides in float32
(every operation rounded) in several summation orders a matrix core or a
kernel may use, on data where the expansion cancels badly (q close to x,
far from the origin), at D up to the library's limit.  CPU only.
"""
import numpy as np
import pytest

U = 2.0 ** -24


def _f32_seq(terms):
    """Sequential float32 sum over axis 1 (every addition rounded)."""
    acc = np.zeros(terms.shape[0], dtype=np.float32)
    for j in range(terms.shape[1]):
        acc = (acc + terms[:, j]).astype(np.float32)
    return acc


def _f32_octets(terms):
    """Chunks of 32 dimensions in order; in a chunk four sequential octet
    sums combined as (o0 + o1) + (o2 + o3); chunk sums added in order."""
    n, d = terms.shape
    total = np.zeros(n, dtype=np.float32)
    for c0 in range(0, d, 32):
        octs = []
        for o in range(4):
            lo, hi = c0 + 8 * o, min(c0 + 8 * o + 8, d)
            octs.append(_f32_seq(terms[:, lo:hi]) if lo < hi else np.zeros(n, dtype=np.float32))
        chunk = ((octs[0] + octs[1]).astype(np.float32) + (octs[2] + octs[3]).astype(np.float32)).astype(np.float32)
        total = (total + chunk).astype(np.float32)
    return total


def _f32_ksteps(terms):
    """Products grouped four at a time (the four k indices of one K-step,
    dimensions j0 + s, j0 + 8 + s, j0 + 16 + s, j0 + 24 + s), each group
    summed in float32 and added to a float32 accumulator."""
    n, d = terms.shape
    acc = np.zeros(n, dtype=np.float32)
    for j0 in range(0, d, 32):
        for s in range(8):
            idx = [j for j in (j0 + s, j0 + 8 + s, j0 + 16 + s, j0 + 24 + s) if j < d]
            if idx:
                acc = (acc + _f32_seq(terms[:, idx])).astype(np.float32)
    return acc


def _pairs(kind, d, rng):
    if kind == "normal":
        q = rng.standard_normal((48, d)).astype(np.float32)
        x = rng.standard_normal((48, d)).astype(np.float32)
    elif kind == "cancel":  # near neighbours far from the origin
        base = (1000.0 * rng.standard_normal(d)).astype(np.float32)
        q = (base + 1e-2 * rng.standard_normal((48, d))).astype(np.float32)
        x = (base + 1e-2 * rng.standard_normal((48, d))).astype(np.float32)
    elif kind == "integer":
        q = rng.integers(-8, 9, (48, d)).astype(np.float32)
        x = rng.integers(-8, 9, (48, d)).astype(np.float32)
    else:  # mixed scales per dimension
        sc = np.exp(3.0 * rng.standard_normal(d)).astype(np.float32)
        q = (sc * rng.standard_normal((48, d))).astype(np.float32)
        x = (sc * rng.standard_normal((48, d))).astype(np.float32)
    return q, x


@pytest.mark.parametrize("kind", ["normal", "cancel", "integer", "scales"])
@pytest.mark.parametrize("d", [32, 100, 960, 4096])
def test_expanded_form_within_margin(kind, d):
    rng = np.random.default_rng(d * 7 + len(kind))
    q, x = _pairs(kind, d, rng)
    diff = (q - x).astype(np.float32)
    sq = (diff * diff).astype(np.float32)
    reported = [_f32_octets(sq), _f32_seq(sq)]  # fixed-order sums the exact paths may use
    qq = (q * q).astype(np.float32)
    xx = (x * x).astype(np.float32)
    qx = (q * x).astype(np.float32)
    norms64 = (q.astype(np.float64) ** 2).sum(1) + (x.astype(np.float64) ** 2).sum(1)
    e = 4.0 * (d + 64) * U * norms64
    for order in (_f32_seq, _f32_ksteps, _f32_octets):
        nq, nx, dot = order(qq), order(xx), order(qx)
        dp = ((nq + nx).astype(np.float32) - (np.float32(2.0) * dot).astype(np.float32)).astype(np.float32)
        for rep in reported:
            gap = np.abs(dp.astype(np.float64) - rep.astype(np.float64))
            assert np.all(gap <= e), (order.__name__, float((gap / e).max()))


def test_margin_covers_cancellation_but_not_a_distance_relative_one():
    """Where q and x nearly coincide far from the origin the expansion's error
    is far above any margin relative to the distance itself: a margin scaled
    by the distance would drop true neighbours, the norm-scaled one does not."""
    rng = np.random.default_rng(5)
    q, x = _pairs("cancel", 960, rng)
    sq = ((q - x) * (q - x)).astype(np.float32)
    ref = _f32_octets(sq).astype(np.float64)
    nq, nx, dot = _f32_seq((q * q).astype(np.float32)), _f32_seq((x * x).astype(np.float32)), \
        _f32_seq((q * x).astype(np.float32))
    dp = ((nq + nx) - np.float32(2.0) * dot).astype(np.float64)
    gap = np.abs(dp - ref)
    assert np.any(gap > 4.0 * (960 + 64) * U * ref)
    norms64 = (q.astype(np.float64) ** 2).sum(1) + (x.astype(np.float64) ** 2).sum(1)
    assert np.all(gap <= 4.0 * (960 + 64) * U * norms64)
