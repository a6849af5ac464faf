"""GPU parity of the exact path (flat PDX index, linear scan and PDX-BOND)
against the FP64 oracle, through the C ABI.

Sizes span several vectorgroups and wave tiles with ragged tails (n not a
multiple of 64, D not a multiple of the chunk), plus the edge cases of the
method: k = 1, k = 64, k > n, duplicates, a query equal to a row, nq = 0,
D at 1,536 and at its limit 4,096 (no LDS tile),
non-finite queries, and schedule-independence of the result.
"""
import numpy as np
import pytest

import synth
from oracle import exact, layout
from tests.parity import check_knn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pdx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_04422_amd as pdx  # fails loudly if libpdx.so is missing
    return pdx


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _search(pdx, x, q, k, **kw):
    import torch
    ix = pdx.pdx_build(_dev(x), start_rows=kw.pop("start_rows", 0))
    ids, dist = pdx.pdx_search_exact(ix, _dev(q), k, **kw)
    torch.cuda.synchronize()
    return ix, ids.cpu().numpy(), dist.cpu().numpy()


def test_layout_and_means_bit_exact(pdx):
    import torch
    for n, d in [(1, 1), (100, 37), (129, 64), (1000, 130)]:
        x = np.random.default_rng(n + d).standard_normal((n, d)).astype(np.float32)
        print(f"layout n={n} d={d}", flush=True)
        ix = pdx.pdx_build(_dev(x))
        torch.cuda.synchronize()
        ng = (n + 63) // 64
        nb = ng * d * 64 * 4
        mem = ix.mem.cpu().numpy()
        got = mem[:nb].view(np.float32).reshape(ng, d, 64)
        assert np.array_equal(got, layout.to_pdx(x, 64))
        off = (nb + 255) // 256 * 256
        means = mem[off:off + 4 * d].view(np.float32)
        want = layout.column_means_f32(x)
        ulp = np.abs(means.view(np.int32).astype(np.int64) - want.view(np.int32).astype(np.int64))
        assert ulp.max() <= 1


def test_linear_small_config(pdx):
    x, q, _ = synth.workload("linear_10k_d128")
    print("linear 10k x 128, 100 queries", flush=True)
    wi, wd = exact.knn_exact_c(x, q, 10)
    _, gi, gd = _search(pdx, x, q, 10, mode="linear")
    check_knn(x, q, gi, gd, wi, wd)


@pytest.mark.parametrize("layout", ["flat", "buckets"])
@pytest.mark.parametrize("n,d,nq", [(20_001, 100, 300), (9_000, 128, 70), (6_000, 96, 33)])
def test_linear_matrix_tiles_and_tails(pdx, layout, n, d, nq):
    """The matrix-core L2 linear mode: 4 query tiles per wave (nq > 64: 300
    leaves a last wave with two full tiles, a partial one and an empty one;
    70 one wave of 64 and one of 6), one tile per wave (nq <= 64), D not a
    multiple of 32 (a short last sub-chunk), a ragged last vectorgroup, a
    non-finite query, and the bucket layout's padded buckets."""
    import torch
    mix = synth.skewed_mixture(d, 16, 8.0, 4.0, n % 97)
    x, q = mix.data(n), mix.queries(nq)
    q[nq // 2, 3] = np.inf
    print(f"linear matrix {layout} n={n} d={d} nq={nq}", flush=True)
    if layout == "flat":
        ix = pdx.pdx_build(_dev(x))
    else:
        init = torch.arange(0, n, n // 64, device="cuda")[:64]
        ix = pdx.pdx_ivf_build(_dev(x), 64, None, init, kmeans_iters=3)
    ids, dist = pdx.pdx_search_exact(ix, _dev(q), 10, mode="linear")
    torch.cuda.synchronize()
    gi, gd = ids.cpu().numpy(), dist.cpu().numpy()
    assert (gi[nq // 2] == -1).all() and np.isnan(gd[nq // 2]).all()
    keep = [i for i in range(nq) if i != nq // 2]
    wi, wd = exact.knn_exact_c(x, q[keep], 10)
    check_knn(x, q[keep], gi[keep], gd[keep], wi, wd)


@pytest.mark.parametrize("mode", ["linear", "bond"])
@pytest.mark.parametrize("n,d,k", [(3001, 100, 10), (4096, 37, 1), (1000, 64, 64), (130, 5, 20)])
def test_integer_inputs_bit_exact(pdx, mode, n, d, k):
    x, q = synth.integer_grid(n, d, 9, lo=-4, hi=4, seed=n + d)
    q[3] = x[17]
    x[n - 1] = x[17]  # duplicate of a row equal to a query
    print(f"integer {mode} n={n} d={d} k={k}", flush=True)
    wi, wd = exact.knn_exact_c(x, q, k)
    _, gi, gd = _search(pdx, x, q, k, mode=mode, start_rows=256)
    check_knn(x, q, gi, gd, wi, wd, exact=True)


def test_bond_skewed_multi_block(pdx):
    x, q, _ = synth.workload("bond_1m_d960", n=40_000, nq=24)
    print("bond skewed 40k x 960", flush=True)
    wi, wd = exact.knn_exact_c(x, q, 10)
    for kw in (dict(), dict(tile_groups=3, queries_per_block=1), dict(chunk=8, queries_per_block=8)):
        _, gi, gd = _search(pdx, x, q, 10, mode="bond", **kw)
        check_knn(x, q, gi, gd, wi, wd)


def test_bond_result_independent_of_schedule(pdx):
    x, q, _ = synth.workload("bond_1m_d960", n=20_000, nq=16)
    print("bond schedule independence", flush=True)
    outs = []
    for kw in (dict(), dict(tile_groups=1, queries_per_block=2), dict(tile_groups=64, queries_per_block=8),
               dict(mode="linear")):
        kw.setdefault("mode", "bond")
        _, gi, gd = _search(pdx, x, q, 10, **kw)
        outs.append((gi, gd))
    for gi, gd in outs[1:3]:
        assert np.array_equal(gi, outs[0][0]) and np.array_equal(gd, outs[0][1])
    # linear mode sums in natural order: same ids up to ties, distances within rounding
    wi, wd = exact.knn_exact_c(x, q, 10)
    check_knn(x, q, outs[3][0], outs[3][1], wi, wd)


def test_k_above_n_and_single_row(pdx):
    x = np.random.default_rng(0).standard_normal((5, 33)).astype(np.float32)
    q = np.random.default_rng(1).standard_normal((3, 33)).astype(np.float32)
    wi, wd = exact.knn_exact_c(x, q, 12)
    for mode in ("linear", "bond"):
        _, gi, gd = _search(pdx, x, q, 12, mode=mode)
        check_knn(x, q, gi, gd, wi, wd)
    _, gi, gd = _search(pdx, x[:1], q, 3, mode="bond")
    assert gi[:, 0].tolist() == [0, 0, 0] and (gi[:, 1:] == -1).all()


def test_zero_queries_and_nonfinite_query(pdx):
    import torch
    x, q = synth.integer_grid(500, 16, 4, seed=3)
    ix = pdx.pdx_build(_dev(x))
    ids, dist = pdx.pdx_search_exact(ix, torch.empty((0, 16), device="cuda"), 5)
    assert ids.shape == (0, 5)
    q[2, 5] = np.nan
    ids, dist = pdx.pdx_search_exact(ix, _dev(q), 5)
    torch.cuda.synchronize()
    gi, gd = ids.cpu().numpy(), dist.cpu().numpy()
    assert (gi[2] == -1).all() and np.isnan(gd[2]).all()
    wi, wd = exact.knn_exact_c(x, q[[0, 1, 3]], 5)
    check_knn(x, q[[0, 1, 3]], gi[[0, 1, 3]], gd[[0, 1, 3]], wi, wd, exact=True)


def test_build_rejects_nonfinite(pdx):
    from paper_2503_04422_amd._lib import PdxError
    x = np.ones((70, 8), dtype=np.float32)
    x[65, 3] = np.inf
    with pytest.raises(PdxError):
        pdx.pdx_build(_dev(x))


def test_full_size_bond_sampled(pdx):
    """1,000,000 x 960, 1,000 queries, in the bench's launch configuration;
    a sample of queries is checked against the oracle one by one."""
    import torch
    x, q, _ = synth.workload("bond_1m_d960")
    print("full size bond 1M x 960 x 1000", flush=True)
    ix = pdx.pdx_build(_dev(x))
    ids, dist = pdx.pdx_search_exact(ix, _dev(q), 10, mode="bond")
    torch.cuda.synchronize()
    gi, gd = ids.cpu().numpy(), dist.cpu().numpy()
    sample = np.random.default_rng(0).choice(q.shape[0], 12, replace=False)
    wi, wd = exact.knn_exact_c(x, q[sample], 10)
    check_knn(x, q[sample], gi[sample], gd[sample], wi, wd)
    # every query: ascending, distinct, valid
    assert (np.diff(gd, axis=1) >= 0).all()
    assert (gi >= 0).all() and (gi < x.shape[0]).all()


@pytest.mark.parametrize("mode", ["bond", "linear"])
def test_tile_path_ties_overflow_and_fallback(pdx, mode):
    """All rows tie with the queries: every vector survives, the LDS survivor
    queue and the per-query candidate buffer overflow (in linear mode the
    matrix-core listing pass's list), and the group-path fallback must still
    return the k lowest ids (distance 0)."""
    x = np.zeros((20_000, 64), dtype=np.float32)
    x[::7, 3] = 1.0
    q = np.zeros((70, 64), dtype=np.float32)
    print(f"tile path overflow {mode}", flush=True)
    wi, wd = exact.knn_exact_c(x, q, 10)
    _, gi, gd = _search(pdx, x, q, 10, mode=mode, start_rows=256)
    check_knn(x, q, gi, gd, wi, wd, exact=True)


def test_tile_path_binary_ties(pdx):
    x, q = synth.integer_grid(30_000, 64, 40, lo=0, hi=1, seed=21)
    print("tile path binary ties", flush=True)
    wi, wd = exact.knn_exact_c(x, q, 16)
    _, gi, gd = _search(pdx, x, q, 16, mode="bond", start_rows=1000)
    check_knn(x, q, gi, gd, wi, wd, exact=True)


@pytest.mark.parametrize("d", [1536, 4096])
def test_largest_dimensions(pdx, d):
    """D above what one LDS tile holds (1,536) and at PDX_MAX_DIM (4,096):
    both layouts take the vectorgroup path.  Per-dimension scales from 0.1
    to 3 (so the PDX-BOND order matters) and queries near rows (so it
    prunes); L2 linear and PDX-BOND, L1 PDX-BOND and the inner product
    against the oracle, flat and bucket layouts."""
    from tests.parity import check_knn_metric
    rng = np.random.default_rng(d)
    scale = np.linspace(0.1, 3.0, d)
    x = (rng.standard_normal((3000, d)) * scale).astype(np.float32)
    q = (x[rng.choice(3000, 6, replace=False)] + 0.3 * rng.standard_normal((6, d)) * scale).astype(np.float32)
    init = rng.choice(3000, 8, replace=False).astype(np.int64)
    indexes = (("flat", pdx.pdx_build(_dev(x))),
               ("buckets", pdx.pdx_ivf_build(_dev(x), 8, None, _dev(init), kmeans_iters=3)))
    wi, wd = exact.knn_exact_c(x, q, 10)
    for name, ix in indexes:
        for mode in ("linear", "bond"):
            print(f"largest d={d} {name} l2 {mode}", flush=True)
            ids, dist = pdx.pdx_search_exact(ix, _dev(q), 10, mode=mode)
            check_knn(x, q, ids.cpu().numpy(), dist.cpu().numpy(), wi, wd)
        for metric, mode in (("l1", "bond"), ("ip", "linear")):
            print(f"largest d={d} {name} {metric} {mode}", flush=True)
            ids, dist = pdx.pdx_search_exact(ix, _dev(q), 10, mode=mode, metric=metric)
            mi, md = exact.knn_exact(x, q, 10, metric=metric)
            check_knn_metric(x, q, ids.cpu().numpy(), dist.cpu().numpy(), mi, md, metric)
