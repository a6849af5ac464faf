"""Pins for the low-precision storage oracle.  CPU only.

* hand-worked codes of both formats;
* the encoders equal torch's CPU conversions (a library routine) on random
  values inside the formats' ranges, and a planted one-bit rounding mistake
  is caught;
* decode error bounds (unit roundoff of the format: 8 significant bits for
  bfloat16, 4 for e4m3): |x - bf16(x)| <= 2^-8 |x|; e4m3 relative error
  <= 2^-4 in the normal range;
* fp8 scales, codes and decoded values pinned by value on a hand-worked
  matrix (tests/golden/hand_fp8_scales.json); a planted divisor of 240
  (another 8-bit format's largest value) is caught;
* the rerank reference keeps the exact top-k when r covers every row, and a
  hand-worked case (tests/golden/hand_rerank.json) pins the first stage's
  ranking, its cut at r and its ties: a planted first stage ranked by the
  exact distance, or cut at r + 1, is caught.
"""
import numpy as np
import pytest
import torch

from oracle import exact, lowp
from tests.conftest import golden

HAND_BF16 = [(1.0, 0x3F80), (-2.0, 0xC000), (1.00390625, 0x3F80),   # tie 1 + 2^-8 -> even (down)
             (1.01171875, 0x3F82), (3.140625, 0x4049), (0.0, 0x0000)]
HAND_E4M3 = [(1.0, 0x38), (448.0, 0x7E), (500.0, 0x7E), (-1.5, 0xBC), (2.0 ** -9, 0x01),
             (2.0 ** -6, 0x08), (1.0625, 0x38),                       # tie 1 + 1/16 -> even (down)
             (1.1875, 0x3A), (0.0, 0x00), (3 * 2.0 ** -10, 0x02)]      # tie 1.5 * 2^-9 -> 2 * 2^-9


@pytest.mark.parametrize("v,code", HAND_BF16)
def test_bf16_hand(v, code):
    assert int(lowp.bf16_encode(np.array([v], np.float32))[0]) == code


@pytest.mark.parametrize("v,code", HAND_E4M3)
def test_e4m3_hand(v, code):
    assert int(lowp.e4m3_encode(np.array([v], np.float32))[0]) == code


def test_bf16_matches_torch_and_bound():
    x = np.random.default_rng(0).standard_normal(200_000).astype(np.float32) * np.float32(3.7)
    got = lowp.bf16_encode(x)
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, want)
    dec = lowp.bf16_decode(got).astype(np.float64)
    assert np.all(np.abs(dec - x) <= 2.0 ** -8 * np.abs(x))


def test_e4m3_matches_torch_and_bound():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 20_000), rng.standard_normal(20_000) * 0.01,
                        rng.standard_normal(5_000) * 1e-3]).astype(np.float32)
    got = lowp.e4m3_encode(x)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(got, want)
    dec = lowp.e4m3_decode(got).astype(np.float64)
    normal = np.abs(x) >= 2.0 ** -6
    assert np.all(np.abs(dec - x)[normal] <= 2.0 ** -4 * np.abs(x[normal]))
    # decode inverts encode on every finite code
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    assert np.array_equal(lowp.e4m3_encode(lowp.e4m3_decode(codes)), codes)
    # a planted mistake (truncation instead of rounding) disagrees with the library
    trunc = np.array([np.float32(1.1) ], np.float32)
    assert int(lowp.e4m3_encode(trunc)[0]) != 0x38  # 1.1 rounds up to 1.125 (0x39), not down


def test_fp8_scaled_round_trip():
    rng = np.random.default_rng(2)
    x = (rng.standard_normal((500, 24)) * rng.uniform(0.01, 5, 24)[None, :]).astype(np.float32)
    x[:, 5] = 0.0
    s = lowp.fp8_scales(x)
    assert s[5] == 1.0
    codes = lowp.fp8_encode(x, s)
    dec = lowp.fp8_decode(codes, s)
    assert np.abs(codes.astype(np.int32) & 0x7F).max() <= 0x7E
    big = np.abs(x) >= (2.0 ** -6) * s[None, :]
    assert np.all(np.abs(dec - x)[big] <= 2.0 ** -4 * np.abs(x[big]) * 1.0001)
    assert np.all(dec[:, 5] == 0)


def test_rerank_full_r_is_exact():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((300, 16)).astype(np.float32)
    xa = lowp.bf16_decode(lowp.bf16_encode(x))
    q = rng.standard_normal(16).astype(np.float32)
    ids, dist = lowp.rerank(x, xa, np.arange(300), q, 10, 300)
    wi, wd = exact.knn_exact(x, q[None], 10)
    assert ids.tolist() == wi[0].tolist()
    np.testing.assert_allclose(dist, wd[0], rtol=1e-12)


def test_fp8_scales_hand_worked():
    g = golden("hand_fp8_scales.json")
    x = np.array(g["x"], np.float32)
    s = lowp.fp8_scales(x)
    assert s.dtype == np.float32 and s.tolist() == g["scales"]
    codes = lowp.fp8_encode(x, s)
    assert codes.tolist() == g["codes"]
    assert lowp.fp8_decode(codes, s).tolist() == g["decoded"]
    # a planted divisor of 240 instead of 448 gives other scales; the codes
    # alone would not show it (the largest value saturates either way)
    planted = (np.abs(x).max(axis=0) / np.float32(240.0)).astype(np.float32)
    planted[np.abs(x).max(axis=0) == 0] = 1.0
    assert planted.tolist() != g["scales"]


def _rerank_exact_first(x_exact, x_approx, rows, q, k, r):
    """A planted mistake: the first stage ranks by the exact distance."""
    return lowp.rerank(x_exact, x_exact, rows, q, k, r)


def test_rerank_hand_worked():
    g = golden("hand_rerank.json")
    xe = np.array(g["exact"], np.float32)
    xa = np.array(g["approx"], np.float32)
    q = np.array(g["query"], np.float32)
    rows = np.arange(xe.shape[0])
    for c in g["cases"]:
        ids, dist = lowp.rerank(xe, xa, rows, q, c["k"], c["r"])
        assert ids.tolist() == c["ids"], c
        assert dist.tolist() == [float(v) for v in c["dist"]], c
    # planted mistakes disagree with the hand-worked cases
    c = g["cases"][0]
    assert _rerank_exact_first(xe, xa, rows, q, c["k"], c["r"])[0].tolist() != c["ids"]
    assert lowp.rerank(xe, xa, rows, q, c["k"], c["r"] + 1)[0].tolist() != c["ids"]


def test_e4m3_array_encoding_equals_the_scalar_one():
    """The whole-array encoder takes the scalar encoder's steps: equal codes
    on every e4m3 code's value, the midpoints between neighbouring codes
    (ties to even), values nudged either side of them, subnormals, zeros of
    both signs, saturation, and random values over the whole range."""
    codes = np.arange(256, dtype=np.uint8)
    codes = codes[(codes & 0x7F) != 0x7F]  # no NaN codes
    vals = lowp.e4m3_decode(codes).astype(np.float64)
    pos = np.unique(vals[vals > 0])
    mids = (pos[:-1] + pos[1:]) / 2
    probe = np.concatenate([vals, mids, -mids, np.nextafter(mids.astype(np.float32), np.float32(0)),
                            np.nextafter(mids.astype(np.float32), np.float32(np.inf)),
                            [0.0, -0.0, 448.0, 449.0, 464.0, 1e6, -1e6, 2.0 ** -10, 2.0 ** -11, 3 * 2.0 ** -11]])
    rng = np.random.default_rng(5)
    probe = np.concatenate([probe, rng.standard_normal(20_000) * 2.0 ** rng.integers(-12, 10, 20_000)])
    probe = probe.astype(np.float32)
    assert np.array_equal(lowp.e4m3_encode_array(probe), lowp.e4m3_encode(probe))
    x = rng.standard_normal((300, 24)).astype(np.float32) * 3
    s = lowp.fp8_scales(x)
    assert np.array_equal(lowp.fp8_encode_array(x, s), lowp.fp8_encode(x, s))
