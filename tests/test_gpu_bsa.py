"""BSA's test inside IVF (bound 3: error quantiles from the Cauchy-Schwarz
inequality with a multiplier m, Section 2.3) on the GPU against the FP64
oracle (oracle.pdxearch.bsa_ivf_search, pinned by hand-worked thresholds
and by equality with IVF-flat at m = 1), through the C ABI.

* m = 1 makes the estimate a lower bound: the search equals the oracle's
  IVF-flat (index parts from the oracle, passed in) under the tie rule, on
  the one-query and batched vector-ALU scans, on integer data bit for bit,
  while pruning (fewer values evaluated than IVF-flat);
* m < 1: recall against IVF-flat within 0.02 of the oracle's sequential
  BSA search with the same m (the result depends on the order in which the
  threshold tightens, so per-query ids are not pinned);
* a PCA index (BSA's projection) with m = 1 over every bucket is exact;
* argument errors: the matrix-core engine, another delta_d, m outside
  [0, 1].
"""
import ctypes

import numpy as np
import pytest

import synth
from oracle import exact, kmeans, pdxearch as px, rotation
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


def _oracle_index(x, nlist, seed, rotate=True, iters=6):
    d = x.shape[1]
    r32 = (rotation.orthogonal_from_gaussian(np.random.default_rng(seed).standard_normal((d, d))).astype(np.float32)
           if rotate else np.eye(d, dtype=np.float32))
    xr = rotation.rotate_rows(x, r32.astype(np.float64))
    init = np.random.default_rng(seed + 1).choice(x.shape[0], nlist, replace=False)
    c, lab, _ = kmeans.lloyd(xr, init, iters)
    return r32, xr, c.astype(np.float32), lab


def _probe_tied(c, qr, nprobe):
    dist = np.sort(exact.sqdist(c, qr))
    return nprobe < dist.size and abs(dist[nprobe] - dist[nprobe - 1]) <= 1e-5 * dist[nprobe]


def _build(pdx, x, r32, c, lab):
    return pdx.pdx_ivf_build(_dev(x), c.shape[0], None, None, rotation=_dev(r32), centroids=_dev(c),
                             assign=_dev(lab.astype(np.int32)))


@pytest.mark.parametrize("qpw", [1, 4])
def test_m_one_equals_ivf_flat_and_prunes(pdx, qpw):
    import torch
    mix = synth.skewed_mixture(256, 24, 32.0, 4.0, 9)
    x = mix.data(20_000)
    q = mix.queries(40, 91)
    nlist, k = 32, 10
    r32, xr, c, lab = _oracle_index(x, nlist, 4)
    lists = kmeans.lists_from_labels(lab, nlist)
    ix = _build(pdx, x, r32, c, lab)
    qr = rotation.rotate_rows(q, r32.astype(np.float64))
    print(f"bsa m=1 parity queries_per_wave={qpw}", flush=True)
    for nprobe in (1, 4, nlist):
        cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
        gi, gd = pdx.pdx_search_ivf(ix, _dev(q), k, nprobe, bound="bsa", bsa_m=1.0, queries_per_wave=qpw,
                                    engine=1, counters=cnt)
        gi, gd = _np(gi), _np(gd)
        keep = [i for i in range(q.shape[0]) if not _probe_tied(c, qr[i], nprobe)]
        want = [px.ivf_flat(xr, lists, c, qr[i], k, nprobe) for i in keep]
        check_knn(xr, qr[keep], gi[keep], gd[keep], np.stack([w[0] for w in want]), np.stack([w[1] for w in want]))
        if nprobe > 1:
            full = torch.zeros(4, dtype=torch.int64, device="cuda")
            pdx.pdx_search_ivf(ix, _dev(q), k, nprobe, eps0=float("inf"), queries_per_wave=qpw, engine=1,
                               counters=full)
            assert int(cnt[2]) < int(_np(full)[2]), "BSA's bound pruned nothing"


def test_m_one_integer_inputs_bit_exact(pdx):
    x, q = synth.integer_grid(6000, 128, 24, -6, 6, seed=12)
    nlist, k = 16, 10
    r32, xr, c, lab = _oracle_index(x, nlist, 5, rotate=False)
    c = np.rint(c).astype(np.float32)  # integer centroids: every distance exact
    lab = np.array([int(np.argmin(exact.sqdist(c, v))) for v in x])
    lists = kmeans.lists_from_labels(lab, nlist)
    ix = _build(pdx, x, r32, c, lab)
    for nprobe in (1, 5, nlist):
        gi, gd = pdx.pdx_search_ivf(ix, _dev(q), k, nprobe, bound="bsa", bsa_m=1.0, engine=1)
        gi, gd = _np(gi), _np(gd)
        for i in range(q.shape[0]):
            if _probe_tied(c, q[i].astype(np.float64), nprobe):
                continue
            wi, wd = px.ivf_flat(x, lists, c, q[i], k, nprobe)
            assert gi[i].tolist() == wi.tolist(), (nprobe, i)
            assert gd[i].astype(np.float64).tolist() == wd.tolist()


@pytest.mark.parametrize("m", [0.9, 0.75])
def test_m_below_one_recall_band(pdx, m):
    mix = synth.skewed_mixture(256, 24, 32.0, 4.0, 10)
    x = mix.data(20_000)
    q = mix.queries(80, 92)
    nlist, k, nprobe = 32, 10, 6
    r32, xr, c, lab = _oracle_index(x, nlist, 6)
    lists = kmeans.lists_from_labels(lab, nlist)
    ix = _build(pdx, x, r32, c, lab)
    qr = rotation.rotate_rows(q, r32.astype(np.float64))
    print(f"bsa recall band m={m}", flush=True)
    flat = np.stack([px.ivf_flat(xr, lists, c, v, k, nprobe)[0] for v in qr])
    seq = np.stack([px.bsa_ivf_search(xr, lists, c, v, k, nprobe, m)[0] for v in qr])
    for qpw in (1, 4):
        gi, _ = pdx.pdx_search_ivf(ix, _dev(q), k, nprobe, bound="bsa", bsa_m=m, queries_per_wave=qpw, engine=1)
        r_gpu = exact.recall_at_k(flat, _np(gi))
        r_seq = exact.recall_at_k(flat, seq)
        assert abs(r_gpu - r_seq) <= 0.02, (qpw, r_gpu, r_seq)


def test_pca_index_with_bsa_is_exact_over_all_buckets(pdx):
    import torch
    mix = synth.skewed_mixture(128, 16, 32.0, 4.0, 11)
    x = mix.data(10_000)
    q = mix.queries(24, 93)
    nlist = 10
    init = np.random.default_rng(2).choice(x.shape[0], nlist, replace=False).astype(np.int64)
    ix = pdx.pdx_ivf_build(_dev(x), nlist, None, _dev(init), kmeans_iters=4, rotation_kind="pca")
    gi, gd = pdx.pdx_search_ivf(ix, _dev(q), 10, nlist, bound="bsa", bsa_m=1.0)
    torch.cuda.synchronize()
    wi, wd = exact.knn_exact(x, q, 10)
    check_knn(x, q, _np(gi), _np(gd), wi, wd)


def test_bsa_argument_errors(pdx):
    from paper_2503_04422_amd import _lib
    mix = synth.skewed_mixture(128, 8, 32.0, 4.0, 12)
    x = mix.data(2000)
    q = _dev(mix.queries(4, 94))
    init = np.arange(4, dtype=np.int64) * 100
    ix = pdx.pdx_ivf_build(_dev(x), 4, None, _dev(init), kmeans_iters=2)
    for kw, status in (({"engine": 2}, _lib.PDX_EUNSUPPORTED), ({"delta_d": 64}, _lib.PDX_EUNSUPPORTED),
                       ({"bsa_m": 1.5}, _lib.PDX_EINVAL)):
        with pytest.raises(_lib.PdxError) as ei:
            pdx.pdx_search_ivf(ix, q, 10, 2, bound="bsa", **kw)
        assert ei.value.status == status, kw
