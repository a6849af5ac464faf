"""GPU parity of the L1 and inner-product exact searches against the FP64
oracle, through the C ABI.

* L1 (linear and PDX-BOND, flat and bucket layouts): integer inputs bit for
  bit (sums of small integers are exact in float32), real inputs under the
  relative 1e-5 rule;
* inner product (linear, matrix cores): integer inputs bit for bit, real
  inputs within 1e-5 |q| max|v|, ragged D (not a multiple of 4 or 32),
  bucket layouts with and without rotation (a rotation preserves inner
  products), k > n, non-finite queries, nq = 0, and the full 1M x 960
  workload on sampled queries;
* errors: the inner product with PDX-BOND, an unknown metric.
"""
import numpy as np
import pytest

import synth
from oracle import exact
from tests.parity import check_knn_metric

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


def _buckets(pdx, x, nlist, seed, gaussian=None):
    init = np.random.default_rng(seed).choice(x.shape[0], nlist, replace=False).astype(np.int64)
    return pdx.pdx_ivf_build(_dev(x), nlist, None if gaussian is None else _dev(gaussian), _dev(init),
                             kmeans_iters=4)


@pytest.mark.parametrize("layout", ["flat", "buckets"])
@pytest.mark.parametrize("n,d,k", [(3001, 96, 10), (2000, 37, 64), (130, 5, 20)])
def test_integer_inputs_bit_exact(pdx, layout, n, d, k):
    x, q = synth.integer_grid(n, d, 9, lo=-4, hi=4, seed=n + 7 * d)
    q[2] = x[11]
    x[n - 1] = x[11]
    ix = pdx.pdx_build(_dev(x)) if layout == "flat" else _buckets(pdx, x, 7, n)
    for metric, modes in (("l1", ("linear", "bond")), ("ip", ("linear",))):
        for mode in modes:
            print(f"integer {metric} {mode} {layout} n={n} d={d} k={k}", flush=True)
            gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), k, mode=mode, metric=metric))
            wi, wd = exact.knn_exact(x, q, k, metric=metric)
            check_knn_metric(x, q, gi, gd, wi, wd, metric, exact=True)


@pytest.mark.parametrize("layout", ["flat", "buckets"])
def test_real_inputs(pdx, layout):
    x, q, _ = synth.workload("bond_1m_d960", n=20_000, nq=24)
    x, q = x[:, :200].copy(), q[:, :200].copy()
    ix = pdx.pdx_build(_dev(x)) if layout == "flat" else _buckets(pdx, x, 32, 3)
    for metric, mode in (("l1", "bond"), ("l1", "linear"), ("ip", "linear")):
        print(f"real {metric} {mode} {layout}", flush=True)
        gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, mode=mode, metric=metric))
        wi, wd = exact.knn_exact(x, q, 10, metric=metric)
        check_knn_metric(x, q, gi, gd, wi, wd, metric)


@pytest.mark.parametrize("d", [37, 100, 130])
def test_inner_product_ragged_dimensions(pdx, d):
    rng = np.random.default_rng(d)
    x = rng.standard_normal((5000, d)).astype(np.float32)
    q = rng.standard_normal((70, d)).astype(np.float32)  # 70: a partly filled query block
    print(f"ip ragged d={d}", flush=True)
    ix = pdx.pdx_build(_dev(x))
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 16, mode="linear", metric="ip"))
    wi, wd = exact.knn_exact(x, q, 16, metric="ip")
    check_knn_metric(x, q, gi, gd, wi, wd, "ip")


def test_inner_product_rotated_buckets(pdx):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((8000, 128)).astype(np.float32)
    q = rng.standard_normal((20, 128)).astype(np.float32)
    print("ip rotated buckets", flush=True)
    ix = _buckets(pdx, x, 16, 6, gaussian=rng.standard_normal((128, 128)))
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, mode="linear", metric="ip"))
    wi, wd = exact.knn_exact(x, q, 10, metric="ip")
    check_knn_metric(x, q, gi, gd, wi, wd, "ip")


def test_edges_and_errors(pdx):
    import torch
    from paper_2503_04422_amd._lib import PdxError
    x, q = synth.integer_grid(40, 32, 4, seed=8)
    q[1, 2] = np.nan
    ix = pdx.pdx_build(_dev(x))
    for metric, mode in (("ip", "linear"), ("l1", "bond")):
        print(f"edges {metric}", flush=True)
        gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 50, mode=mode, metric=metric))
        assert (gi[1] == -1).all() and np.isnan(gd[1]).all()
        keep = [0, 2, 3]
        wi, wd = exact.knn_exact(x, q[keep], 50, metric=metric)
        check_knn_metric(x, q[keep], gi[keep], gd[keep], wi, wd, metric, exact=True)
        ids, _ = pdx.pdx_search_exact(ix, torch.empty((0, 32), device="cuda"), 5, mode=mode, metric=metric)
        assert ids.shape == (0, 5)
    with pytest.raises(PdxError):
        pdx.pdx_search_exact(ix, _dev(q), 5, mode="bond", metric="ip")
    # an unknown metric through the C ABI
    import ctypes
    from paper_2503_04422_amd import _lib
    p = _lib.pdx_search_params(_lib.PDX_MODE_LINEAR, 0, 0, 0, None, None, 7)
    qd = _dev(q)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    ids = torch.empty((4, 5), dtype=torch.int64, device="cuda")
    dist = torch.empty((4, 5), dtype=torch.float32, device="cuda")
    st = _lib.lib.pdx_search_exact(ix.handle, qd.data_ptr(), 4, 5, ctypes.byref(p), ws.data_ptr(), ws.numel(),
                                   ids.data_ptr(), dist.data_ptr(), None)
    assert st == _lib.PDX_EINVAL and b"metric" in _lib.lib.pdx_last_error()


def test_inner_product_full_size_sampled(pdx):
    """1,000,000 x 960, 1,000 queries, the bench's default workload."""
    x, q, _ = synth.workload("bond_1m_d960")
    print("ip full size 1M x 960 x 1000", flush=True)
    ix = pdx.pdx_build(_dev(x))
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, mode="linear", metric="ip"))
    sample = np.random.default_rng(0).choice(q.shape[0], 8, replace=False)
    wi, wd = exact.knn_exact_blocked(x, q[sample], 10, metric="ip")
    check_knn_metric(x, q[sample], gi[sample], gd[sample], wi, wd, "ip")
    assert (np.diff(gd, axis=1) >= 0).all()
    assert (gi >= 0).all() and (gi < x.shape[0]).all()


@pytest.mark.parametrize("layout", ["flat", "buckets"])
@pytest.mark.parametrize("d", [128, 960])
def test_l1_tile_path(pdx, layout, d):
    """L1 with PDX-BOND at D a multiple of 32 (the bucket layout's LDS-tile
    path with the L1 centroid bound; the flat layout's vectorgroup path):
    real inputs under the relative 1e-5 rule, and a tie-heavy case whose
    candidate buffers overflow on the bucket layout (the L1 fallback path),
    bit for bit."""
    x, q, _ = synth.workload("bond_1m_d960", n=12_000, nq=20)
    x, q = x[:, :d].copy(), q[:, :d].copy()
    ix = pdx.pdx_build(_dev(x)) if layout == "flat" else _buckets(pdx, x, 24, d)
    print(f"l1 tile path {layout} d={d}", flush=True)
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, mode="bond", metric="l1"))
    wi, wd = exact.knn_exact(x, q, 10, metric="l1")
    check_knn_metric(x, q, gi, gd, wi, wd, "l1")
    z = np.zeros((8_000, d), dtype=np.float32)
    z[::5, 3] = 1.0
    qz = np.zeros((6, d), dtype=np.float32)
    iz = pdx.pdx_build(_dev(z)) if layout == "flat" else _buckets(pdx, z, 8, 5)
    print(f"l1 tile path overflow {layout} d={d}", flush=True)
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(iz, _dev(qz), 10, mode="bond", metric="l1"))
    wi, wd = exact.knn_exact(z, qz, 10, metric="l1")
    check_knn_metric(z, qz, gi, gd, wi, wd, "l1", exact=True)


@pytest.mark.parametrize("d", [128, 960])
def test_inner_product_tile_path(pdx, d):
    """Inner product on the bucket layout with D a multiple of 32 (the tile
    path with the Cauchy-Schwarz tile bound): real inputs, rotated and
    unrotated, under the 1e-5 |q| max|v| rule; integer inputs bit for bit;
    a tie-heavy case whose candidate buffers overflow (the full-scan
    fallback); k above the bucket sizes."""
    x, q, _ = synth.workload("bond_1m_d960", n=12_000, nq=20)
    x, q = x[:, :d].copy(), q[:, :d].copy()
    for gauss in (None, np.random.default_rng(d).standard_normal((d, d))):
        print(f"ip tile path d={d} rotated={gauss is not None}", flush=True)
        ix = _buckets(pdx, x, 24, d, gaussian=gauss)
        gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, mode="linear", metric="ip"))
        wi, wd = exact.knn_exact(x, q, 10, metric="ip")
        check_knn_metric(x, q, gi, gd, wi, wd, "ip")
    xi, qi = synth.integer_grid(5000, d, 12, lo=-4, hi=4, seed=d)
    qi[3] = xi[17]
    ixi = _buckets(pdx, xi, 16, 7)
    print(f"ip tile path integer d={d}", flush=True)
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ixi, _dev(qi), 10, mode="linear", metric="ip"))
    wi, wd = exact.knn_exact(xi, qi, 10, metric="ip")
    check_knn_metric(xi, qi, gi, gd, wi, wd, "ip", exact=True)
    z = np.zeros((12_000, d), dtype=np.float32)
    z[::2, 5] = 1.0  # 6,000 rows tie for the best score: more than a candidate buffer holds
    qz = np.zeros((5, d), dtype=np.float32)
    qz[:, 5] = 1.0
    iz = _buckets(pdx, z, 6, 3)
    print(f"ip tile path overflow d={d}", flush=True)
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(iz, _dev(qz), 10, mode="linear", metric="ip"))
    wi, wd = exact.knn_exact(z, qz, 10, metric="ip")
    check_knn_metric(z, qz, gi, gd, wi, wd, "ip", exact=True)
    x2, q2 = synth.integer_grid(40, 32 if d == 128 else 64, 3, seed=9)
    ix2 = _buckets(pdx, x2, 3, 2)
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix2, _dev(q2), 50, mode="linear", metric="ip"))
    wi, wd = exact.knn_exact(x2, q2, 50, metric="ip")
    check_knn_metric(x2, q2, gi, gd, wi, wd, "ip", exact=True)
