"""GPU parity of the low-precision IVF search's re-rank of more than 64
candidates (rerank R > PDX_MAX_K: the per-query candidate buffer) against
the oracle (oracle.lowp.rerank: the R best of the probed rows by the
decoded distance, then the k best of those by the exact distance).

* eps0 = inf: the GPU returns the oracle's ids and exact distances (tie
  rule 1e-5) wherever the R-th and next decoded distances are not tied at
  the rounding level (elsewhere a result valid for either candidate set),
  for R = 100 and 1000 on FP8 and R = 4096 on BF16 (the "top 4K" of the
  5M x 768 low-precision workload), and for R above the probed rows (every
  probed row a candidate);
* a buffer far smaller than the probed rows (many compaction and resume
  rounds) gives the same bits as the default buffer, at eps0 = inf;
* eps0 = 2.1: recall against f32 IVF-flat and exact distances;
* a non-finite query gets a NaN row; argument errors.
"""
import numpy as np
import pytest

import synth
from oracle import exact, kmeans, lowp, pdxearch as px
from tests.parity import check_knn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pdx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_04422_amd as pdx
    return pdx


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _setup(pdx, n, d, nlist, nq, seed, lowp_kinds):
    mix = synth.anisotropic_unit_mixture(d, 16, seed)
    x = mix.data(n)
    q = mix.queries(nq)
    init = np.random.default_rng(seed + 1).choice(n, nlist, replace=False)
    c, lab, _ = kmeans.lloyd(x, init, 5)
    c32 = c.astype(np.float32)
    lists = kmeans.lists_from_labels(lab, nlist)
    ix = pdx.pdx_ivf_build(_dev(x), nlist, None, None, lowp=lowp_kinds, centroids=_dev(c32),
                           assign=_dev(lab.astype(np.int32)))
    dec = {}
    if "bf16" in lowp_kinds:
        dec["bf16"] = lowp.bf16_decode(lowp.bf16_encode(x))
    if "fp8" in lowp_kinds:
        s = lowp.fp8_scales(x)
        dec["fp8"] = lowp.fp8_decode(lowp.fp8_encode(x, s), s)
    return dict(x=x, q=q, c32=c32, lists=lists, ix=ix, dec=dec)


@pytest.fixture(scope="module")
def small(pdx):
    return _setup(pdx, 12_000, 96, 24, 32, 21, ("bf16", "fp8"))


@pytest.fixture(scope="module")
def big(pdx):
    return _setup(pdx, 40_000, 64, 16, 24, 22, ("bf16",))


def _probed_rows(st, qv, nprobe):
    probe = px.ivf_probe_order(st["c32"], qv.astype(np.float64), nprobe)
    return np.concatenate([st["lists"][p] for p in probe])


def _check_rerank(st, dtype, r, nprobe, gi, gd, min_exact, band=1e-5):
    """Oracle parity where the R-th and next decoded distances are apart;
    where they are tied at the scan's rounding level (relative `band`) the
    candidate set lies between the rows surely in (decoded distance below a
    band of twice that width around the R-th) and those possibly in (at or
    below the band's top), so: every returned id is possibly in, distances
    are exact, and the k-th distance lies between the k-th of the exact
    top-k of the two sets."""
    xd = st["dec"][dtype]
    exact_checked = 0
    for i in range(st["q"].shape[0]):
        qv = st["q"][i]
        rows = _probed_rows(st, qv, nprobe)
        ad = exact.sqdist(xd[rows], qv)
        approx = np.sort(ad)
        if approx.size > r and abs(approx[r] - approx[r - 1]) <= band * approx[r]:
            lo, hi = approx[r - 1] * (1 - 2 * band), approx[r - 1] * (1 + 2 * band)
            sure, maybe = rows[ad < lo], rows[ad <= hi]
            assert np.all(np.isin(gi[i], maybe)), i
            np.testing.assert_allclose(gd[i], exact.sqdist(st["x"][gi[i]], qv), rtol=1e-5)
            _, ws = exact.topk_by_dist_then_id(exact.sqdist(st["x"][sure], qv), sure, 10)
            _, wm = exact.topk_by_dist_then_id(exact.sqdist(st["x"][maybe], qv), maybe, 10)
            assert wm[-1] * (1 - 1e-5) <= gd[i][-1] <= ws[-1] * (1 + 1e-5), i
            continue
        wi, wd = lowp.rerank(st["x"], xd, rows, qv, 10, r)
        check_knn(st["x"], st["q"][i:i + 1], gi[i:i + 1], gd[i:i + 1], wi[None], wd[None])
        exact_checked += 1
    assert exact_checked >= min_exact, exact_checked


@pytest.mark.parametrize("r", [100, 1000])
def test_fp8_wide_rerank_matches_oracle(pdx, small, r):
    st = small
    print(f"wide rerank parity fp8 R={r}", flush=True)
    gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 5, eps0=float("inf"), dtype="fp8", rerank=r)
    _check_rerank(st, "fp8", r, 5, _np(gi), _np(gd), st["q"].shape[0] // 2)


def test_bf16_rerank_4096_matches_oracle(pdx, big):
    st = big
    print("wide rerank parity bf16 R=4096", flush=True)
    gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 4, eps0=float("inf"), dtype="bf16", rerank=4096)
    _check_rerank(st, "bf16", 4096, 4, _np(gi), _np(gd), st["q"].shape[0] // 2)


def test_rerank_above_probed_rows_is_exact(pdx, small):
    """R larger than the probed rows: every probed row is re-ranked, so the
    result is the exact k-NN over the probed buckets."""
    st = small
    gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 2, eps0=float("inf"), dtype="fp8", rerank=8192)
    gi, gd = _np(gi), _np(gd)
    want = [px.ivf_flat(st["x"], st["lists"], st["c32"], v, 10, 2) for v in st["q"]]
    check_knn(st["x"], st["q"], gi, gd, np.stack([w[0] for w in want]), np.stack([w[1] for w in want]))


@pytest.mark.parametrize("dtype,r,cap", [("fp8", 300, 600), ("bf16", 1000, 2000)])
def test_small_buffer_rounds_give_the_same_bits(pdx, small, dtype, r, cap):
    """A buffer of 2R slots against about 2,500 probed rows: queries fill it
    repeatedly and are compacted and resumed; at eps0 = inf the candidate
    set is the R best regardless, so the result is bit-identical."""
    st = small
    print(f"wide rerank rounds {dtype} R={r} capacity={cap}", flush=True)
    gi0, gd0 = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 5, eps0=float("inf"), dtype=dtype, rerank=r)
    gi1, gd1 = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 5, eps0=float("inf"), dtype=dtype, rerank=r,
                                  rerank_capacity=cap, queries_per_wave=1)
    gi0, gd0, gi1, gd1 = _np(gi0), _np(gd0), _np(gi1), _np(gd1)
    assert np.array_equal(gi0, gi1)
    assert np.array_equal(gd0.view(np.int32), gd1.view(np.int32))
    # the workspace grows with the capacity
    ws_small = pdx.pdx_search_ivf_workspace(st["ix"], 32, 10, 5, dtype=dtype, rerank=r, rerank_capacity=cap)
    ws_big = pdx.pdx_search_ivf_workspace(st["ix"], 32, 10, 5, dtype=dtype, rerank=r)
    assert ws_small < ws_big


def test_wide_rerank_pruned_recall_and_nan_query(pdx, big):
    st = big
    q = st["q"].copy()
    q[3, 5] = np.nan
    flat = np.stack([px.ivf_flat(st["x"], st["lists"], st["c32"], v, 10, 6)[0] for v in st["q"]])
    for qpw in (1, 4):
        gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(q), 10, 6, eps0=2.1, dtype="bf16", rerank=4096,
                                    queries_per_wave=qpw)
        gi, gd = _np(gi), _np(gd)
        assert np.all(gi[3] == -1) and np.all(np.isnan(gd[3]))
        keep = [i for i in range(q.shape[0]) if i != 3]
        rec = exact.recall_at_k(flat[keep], gi[keep])
        print(f"bf16 rerank 4096 ads recall vs f32 ivf-flat {rec:.4f} (qpw {qpw})", flush=True)
        assert rec >= 0.97
        for i in keep[::5]:
            ok = gi[i] >= 0
            np.testing.assert_allclose(gd[i][ok], exact.sqdist(st["x"][gi[i][ok]], st["q"][i]), rtol=1e-5)


def test_wide_rerank_argument_errors(pdx, small):
    from paper_2503_04422_amd import _lib
    st = small
    q = _dev(st["q"][:4])
    cases = [({"rerank": _lib.PDX_MAX_RERANK + 1}, _lib.PDX_EUNSUPPORTED),
             ({"rerank": 200, "rerank_capacity": 300}, _lib.PDX_EINVAL),
             ({"rerank": 200, "rerank_capacity": -1}, _lib.PDX_EINVAL)]
    for kw, status in cases:
        with pytest.raises(_lib.PdxError) as ei:
            pdx.pdx_search_ivf(st["ix"], q, 10, 4, dtype="bf16", **kw)
        assert ei.value.status == status, kw


# Matrix cores (engine 2): the scanned distances come from bfloat16 MFMA on
# the codes (|q|^2 + |x|^2 - 2 q.x per 32-dimension sub-chunk), whose
# rounding is wider than the vector ALU's direct sums, so the tie band at
# the R-th candidate is 1e-4.  Vectors a full buffer stopped are resumed on
# the vector ALU.  The ADSampling test every 32 dimensions (whole
# sub-chunks of the codes) keeps these small workloads on the matrix cores.
@pytest.mark.parametrize("dtype,r", [("fp8", 1000), ("bf16", 300)])
def test_matrix_engine_wide_rerank_matches_oracle(pdx, small, dtype, r):
    st = small
    print(f"matrix-core wide rerank parity {dtype} R={r}", flush=True)
    gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 5, eps0=float("inf"), dtype=dtype, rerank=r,
                                engine=2, delta_d=32)
    _check_rerank(st, dtype, r, 5, _np(gi), _np(gd), st["q"].shape[0] // 2, band=1e-4)
    # a buffer of 2R: compaction and resume rounds (resumed on the vector ALU)
    gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 5, eps0=float("inf"), dtype=dtype, rerank=r,
                                engine=2, delta_d=32, rerank_capacity=max(2 * r, r + 256))
    _check_rerank(st, dtype, r, 5, _np(gi), _np(gd), st["q"].shape[0] // 2, band=1e-4)


def test_matrix_engine_rerank_4096(pdx, big):
    st = big
    print("matrix-core wide rerank parity bf16 R=4096", flush=True)
    gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 4, eps0=float("inf"), dtype="bf16", rerank=4096,
                                engine=2, delta_d=32)
    _check_rerank(st, "bf16", 4096, 4, _np(gi), _np(gd), st["q"].shape[0] // 2, band=1e-4)
    q = st["q"].copy()
    q[3, 5] = np.nan
    flat = np.stack([px.ivf_flat(st["x"], st["lists"], st["c32"], v, 10, 6)[0] for v in st["q"]])
    gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(q), 10, 6, eps0=2.1, dtype="bf16", rerank=4096, engine=2,
                                delta_d=32)
    gi, gd = _np(gi), _np(gd)
    assert np.all(gi[3] == -1) and np.all(np.isnan(gd[3]))
    keep = [i for i in range(q.shape[0]) if i != 3]
    rec = exact.recall_at_k(flat[keep], gi[keep])
    print(f"matrix-core bf16 rerank 4096 ads recall vs f32 ivf-flat {rec:.4f}", flush=True)
    assert rec >= 0.97
    for i in keep[::5]:
        ok = gi[i] >= 0
        np.testing.assert_allclose(gd[i][ok], exact.sqdist(st["x"][gi[i][ok]], st["q"][i]), rtol=1e-5)
