"""GPU parity of the low-precision IVF storage (bfloat16, float8 e4m3 with
per-dimension scales) against the oracle.

With no rotation the stored rows are the caller's float32 values, so both
sides encode identical inputs: the codes are compared through the search.
* eps0 = inf, no rerank: the result is the exact top-k over the decoded
  vectors of the probed buckets (f32 accumulation vs the FP64 oracle on the
  oracle's own decoding, tie rule 1e-5).
* eps0 = inf with rerank R: the oracle keeps the R best by decoded distance
  and re-ranks them exactly; the GPU must agree wherever the R-th and next
  candidates are not tied, and its distances are the exact distances.
* the same on the matrix cores with chunks of whole 32-dimension
  sub-chunks, where the codes feed bfloat16 MFMA, at D = 96 and a ragged
  D = 100;
* eps0 = 2.1: recall against f32 IVF-flat stays within the statistical band.
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


@pytest.fixture(scope="module")
def setup(pdx):
    n, d, nlist = 12_000, 96, 24
    mix = synth.anisotropic_unit_mixture(d, 16, 8)
    x = mix.data(n)
    q = mix.queries(48)
    init = np.random.default_rng(9).choice(n, nlist, replace=False)
    c, lab, _ = kmeans.lloyd(x, init, 6)
    c32 = c.astype(np.float32)
    lists = kmeans.lists_from_labels(lab, nlist)
    ix = pdx.pdx_ivf_build(_dev(x), nlist, None, None, lowp=("bf16", "fp8"), centroids=_dev(c32),
                           assign=_dev(lab.astype(np.int32)))
    dec = {"bf16": lowp.bf16_decode(lowp.bf16_encode(x)),
           "fp8": lowp.fp8_decode(lowp.fp8_encode(x, lowp.fp8_scales(x)), lowp.fp8_scales(x))}
    return dict(x=x, q=q, c32=c32, lists=lists, ix=ix, dec=dec, nlist=nlist)


def _probed_rows(st, qv, nprobe):
    probe = px.ivf_probe_order(st["c32"], qv.astype(np.float64), nprobe)
    return np.concatenate([st["lists"][p] for p in probe])


@pytest.mark.parametrize("dtype,engine", [("bf16", 0), ("fp8", 0), ("bf16", 2), ("fp8", 2)])
def test_lowp_scan_exact_over_decoded(pdx, setup, dtype, engine):
    st = setup
    print(f"lowp scan parity {dtype} engine {engine}", flush=True)
    for nprobe in (1, 5):
        gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, nprobe, eps0=float("inf"), dtype=dtype, rerank=-1,
                                    engine=engine)
        gi, gd = _np(gi), _np(gd)
        xd = st["dec"][dtype]
        want = [exact.topk_by_dist_then_id(exact.sqdist(xd[r], st["q"][i]), r, 10)
                for i, r in enumerate(_probed_rows(st, qv, nprobe) for qv in st["q"])]
        check_knn(xd, st["q"], gi, gd, np.stack([w[0] for w in want]), np.stack([w[1] for w in want]))


@pytest.fixture(scope="module")
def ragged(pdx):
    """D = 100: the last 32-dimension sub-chunk holds 4 dimensions."""
    n, d, nlist = 8_000, 100, 16
    mix = synth.anisotropic_unit_mixture(d, 16, 9)
    x = mix.data(n)
    q = mix.queries(40)
    init = np.random.default_rng(10).choice(n, nlist, replace=False)
    c, lab, _ = kmeans.lloyd(x, init, 5)
    c32 = c.astype(np.float32)
    lists = kmeans.lists_from_labels(lab, nlist)
    ix = pdx.pdx_ivf_build(_dev(x), nlist, None, None, lowp=("bf16", "fp8"), centroids=_dev(c32),
                           assign=_dev(lab.astype(np.int32)))
    dec = {"bf16": lowp.bf16_decode(lowp.bf16_encode(x)),
           "fp8": lowp.fp8_decode(lowp.fp8_encode(x, lowp.fp8_scales(x)), lowp.fp8_scales(x))}
    return dict(x=x, q=q, c32=c32, lists=lists, ix=ix, dec=dec, nlist=nlist)


@pytest.mark.parametrize("which,dtype,delta_d", [("setup", "bf16", 32), ("setup", "fp8", 64),
                                                 ("ragged", "bf16", 64), ("ragged", "fp8", 32)])
def test_lowp_matrix_codes_exact_over_decoded(pdx, setup, ragged, which, dtype, delta_d):
    """Matrix cores with chunks of whole 32-dimension sub-chunks: the codes
    go to bfloat16 MFMA (the query as three bfloat16 terms, stored
    sub-chunk norms).  eps0 = inf, no rerank: the exact top-k over the
    decoded vectors of the probed buckets, distances within the tie rule."""
    st = setup if which == "setup" else ragged
    print(f"lowp matrix-code scan parity {which} {dtype} delta_d={delta_d}", flush=True)
    for nprobe, qpw in ((1, 16), (5, 16), (5, 32)):
        gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, nprobe, eps0=float("inf"), dtype=dtype,
                                    rerank=-1, engine=2, delta_d=delta_d, queries_per_wave=qpw)
        gi, gd = _np(gi), _np(gd)
        xd = st["dec"][dtype]
        want = [exact.topk_by_dist_then_id(exact.sqdist(xd[r], st["q"][i]), r, 10)
                for i, r in enumerate(_probed_rows(st, qv, nprobe) for qv in st["q"])]
        check_knn(xd, st["q"], gi, gd, np.stack([w[0] for w in want]), np.stack([w[1] for w in want]))


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_lowp_rerank_matches_oracle(pdx, setup, dtype):
    st = setup
    r = 40
    print(f"lowp rerank parity {dtype}", flush=True)
    gi, gd = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 5, eps0=float("inf"), dtype=dtype, rerank=r)
    gi, gd = _np(gi), _np(gd)
    xd = st["dec"][dtype]
    checked = 0
    for i in range(st["q"].shape[0]):
        rows = _probed_rows(st, st["q"][i], 5)
        approx = np.sort(exact.sqdist(xd[rows], st["q"][i]))
        if approx.size > r and abs(approx[r] - approx[r - 1]) <= 1e-5 * approx[r]:
            continue  # candidate set decided by a rounding-level tie
        wi, wd = lowp.rerank(st["x"], xd, rows, st["q"][i], 10, r)
        check_knn(st["x"], st["q"][i:i + 1], gi[i:i + 1], gd[i:i + 1], wi[None], wd[None])
        checked += 1
    assert checked >= st["q"].shape[0] - 2


def test_lowp_ads_recall_and_errors(pdx, setup):
    from paper_2503_04422_amd._lib import PdxError
    st = setup
    fi, _ = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 6, eps0=float("inf"))
    fi = _np(fi)
    for dtype in ("bf16", "fp8"):
        ai, ad = pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 6, eps0=2.1, dtype=dtype)
        ai, ad = _np(ai), _np(ad)
        rec = exact.recall_at_k(fi, ai)
        print(f"{dtype} ads+rerank recall vs f32 ivf-flat {rec:.4f}", flush=True)
        assert rec >= 0.97
        for i in range(0, st["q"].shape[0], 7):
            ok = ai[i] >= 0
            np.testing.assert_allclose(ad[i][ok], exact.sqdist(st["x"][ai[i][ok]], st["q"][i]), rtol=1e-5)
    from paper_2503_04422_amd._lib import PDX_MAX_RERANK
    with pytest.raises(PdxError):
        pdx.pdx_search_ivf(st["ix"], _dev(st["q"]), 10, 4, dtype="bf16", rerank=PDX_MAX_RERANK + 1)
    x2 = st["x"][:2000]
    ix2 = pdx.pdx_ivf_build(_dev(x2), 4, None, _dev(np.arange(4, dtype=np.int64) * 100), kmeans_iters=2)
    with pytest.raises(PdxError):
        pdx.pdx_search_ivf(ix2, _dev(st["q"]), 10, 2, dtype="fp8")
