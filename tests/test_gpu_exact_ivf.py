"""GPU parity of exact search on the bucket (IVF) layout against the FP64
oracle, through the C ABI.

pdx_search_exact on an index built by pdx_ivf_build visits every vector
(bucket by bucket, START on the query's nearest bucket), so its answer is
the exact k-NN of all rows: integer inputs must match the oracle bit for
bit (unrotated index), real inputs under the tie rule; a rotated index
answers in rotated space.  More than 1,024 queries (two query lists per
tile) for L2, L1 and the inner product.
"""
import numpy as np
import pytest

import synth
from oracle import exact, rotation
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


def _bucket_index(pdx, x, nlist, seed, gaussian=None, iters=4):
    rng = np.random.default_rng(seed)
    init = rng.choice(x.shape[0], nlist, replace=False).astype(np.int64)
    return pdx.pdx_ivf_build(_dev(x), nlist, None if gaussian is None else _dev(gaussian), _dev(init),
                             kmeans_iters=iters)


@pytest.mark.parametrize("mode", ["linear", "bond"])
@pytest.mark.parametrize("n,d,k,nlist", [(3001, 96, 10, 20), (4096, 37, 1, 9), (2000, 64, 64, 7), (130, 5, 20, 3)])
def test_integer_inputs_bit_exact(pdx, mode, n, d, k, nlist):
    x, q = synth.integer_grid(n, d, 9, lo=-4, hi=4, seed=n + d + 1)
    q[3] = x[17]
    x[n - 1] = x[17]
    print(f"bucket layout integer {mode} n={n} d={d} k={k} nlist={nlist}", flush=True)
    ix = _bucket_index(pdx, x, nlist, n)
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), k, mode=mode))
    wi, wd = exact.knn_exact_c(x, q, k)
    check_knn(x, q, gi, gd, wi, wd, exact=True)


def test_bond_skewed_bucket_layout(pdx):
    x, q, _ = synth.workload("bond_1m_d960", n=40_000, nq=24)
    print("bucket layout bond skewed 40k x 960", flush=True)
    ix = _bucket_index(pdx, x, 64, 1)
    wi, wd = exact.knn_exact_c(x, q, 10)
    ref = None
    for kw in (dict(), dict(tile_groups=3, queries_per_block=1), dict(chunk=8, queries_per_block=8),
               dict(start_rows=1), dict(start_rows=1 << 20), dict(rounds=1, dense_min=1),
               dict(rounds=64, dense_min=33), dict(rounds=7, dense_min=16)):
        gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, mode="bond", **kw))
        check_knn(x, q, gi, gd, wi, wd)
        if kw.get("chunk", 32) == 32:  # same summation order: bit-identical across schedules and START sizes
            if ref is None:
                ref = (gi, gd)
            else:
                assert np.array_equal(gi, ref[0]) and np.array_equal(gd, ref[1])


def test_rotated_bucket_layout(pdx):
    x, q, _ = synth.workload("bond_1m_d960", n=20_000, nq=16)
    x, q = x[:, :256].copy(), q[:, :256].copy()
    print("bucket layout rotated 20k x 256", flush=True)
    g = np.random.default_rng(4).standard_normal((256, 256))
    ix = _bucket_index(pdx, x, 32, 2, gaussian=g)
    rot = _np(pdx.pdx_ivf_export(ix)[0]).astype(np.float64)
    xr = rotation.rotate_rows(x, rot)
    qr = rotation.rotate_rows(q, rot)
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, mode="bond"))
    wi, wd = exact.knn_exact(xr, qr, 10)
    check_knn(xr, qr, gi, gd, wi, wd)


def test_bucket_layout_ties_overflow_and_edges(pdx):
    import torch
    x = np.zeros((20_000, 64), dtype=np.float32)
    x[::7, 3] = 1.0
    q = np.zeros((70, 64), dtype=np.float32)
    print("bucket layout overflow", flush=True)
    ix = _bucket_index(pdx, x, 16, 3, iters=2)
    wi, wd = exact.knn_exact_c(x, q, 10)
    for mode in ("bond", "linear"):  # linear: the listing pass overflows into the fallback
        gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, mode=mode))
        check_knn(x, q, gi, gd, wi, wd, exact=True)
    # k above n, a non-finite query, no queries
    x2, q2 = synth.integer_grid(40, 32, 4, seed=8)
    ix2 = _bucket_index(pdx, x2, 3, 4)
    q2[1, 2] = np.inf
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix2, _dev(q2), 50, mode="bond"))
    assert (gi[1] == -1).all() and np.isnan(gd[1]).all()
    keep = [0, 2, 3]
    wi, wd = exact.knn_exact_c(x2, q2[keep], 50)
    check_knn(x2, q2[keep], gi[keep], gd[keep], wi, wd, exact=True)
    ids, _ = pdx.pdx_search_exact(ix2, torch.empty((0, 32), device="cuda"), 5)
    assert ids.shape == (0, 5)


@pytest.mark.parametrize("metric,mode", [("l2", "bond"), ("l1", "bond"), ("ip", "linear")])
def test_more_queries_than_one_list(pdx, metric, mode):
    """1,100 queries on the bucket layout's tile path: more than one
    workgroup's query list holds (1,024), so every tile lists the queries
    that its centroid bound keeps in two passes; each query against the
    oracle."""
    from tests.parity import check_knn_metric
    x, q, _ = synth.workload("bond_1m_d960", n=12_000, nq=1100)
    x, q = x[:, :64].copy(), q[:, :64].copy()
    print(f"bucket layout 1,100 queries {metric} {mode}", flush=True)
    ix = _bucket_index(pdx, x, 24, 13)
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, mode=mode, metric=metric))
    if metric == "l2":
        wi, wd = exact.knn_exact_c(x, q, 10)
        check_knn(x, q, gi, gd, wi, wd)
    else:
        wi, wd = exact.knn_exact(x, q, 10, metric=metric)
        check_knn_metric(x, q, gi, gd, wi, wd, metric)


def test_full_size_bucket_layout_sampled(pdx):
    """1,000,000 x 960, 1,000 queries on 1,024 buckets, in the bench's
    launch configuration; sampled queries against the oracle."""
    x, q, _ = synth.workload("bond_1m_d960")
    print("full size bucket layout 1M x 960 x 1000", flush=True)
    ix = _bucket_index(pdx, x, 1024, 42, iters=20)
    gi, gd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, mode="bond"))
    sample = np.random.default_rng(0).choice(q.shape[0], 12, replace=False)
    wi, wd = exact.knn_exact_c(x, q[sample], 10)
    check_knn(x, q[sample], gi[sample], gd[sample], wi, wd)
    assert (np.diff(gd, axis=1) >= 0).all()
    assert (gi >= 0).all() and (gi < x.shape[0]).all()


def test_exact_tuner_schedules_give_one_answer(pdx):
    """pdx_exact_tune times START block x rounds x dense threshold; every
    schedule returns the same exact answer (bit-identical: the summation
    order per (query, vector) is fixed), the chosen one is the fastest
    measured, and values that cannot change a search are not timed."""
    from paper_2503_04422_amd._lib import PdxError
    x, q, _ = synth.workload("bond_1m_d960", n=40_000, nq=64)
    print("exact tuner 40k x 960, 64 queries", flush=True)
    ix = _bucket_index(pdx, x, 64, 2)
    sched, table = pdx.pdx_exact_tune(ix, _dev(q), 10, reps=1)
    assert len(table) == 27
    assert [(t["start_rows"], t["rounds"], t["dense_min"]) for t in table] == [
        (s, r, m) for s in (64, 128, 256) for r in (2, 4, 8) for m in (4, 8, 16)]
    assert all(t["ms"] >= 0 for t in table)  # bucket layout, L2 BOND: every value matters
    best = min(table, key=lambda t: t["ms"])
    assert sched == {kk: best[kk] for kk in ("start_rows", "rounds", "dense_min")}
    ri, rd = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10))
    ti, td = (_np(t) for t in pdx.pdx_search_exact(ix, _dev(q), 10, **sched))
    assert np.array_equal(ri, ti) and np.array_equal(rd, td)
    wi, wd = exact.knn_exact_c(x, q, 10)
    check_knn(x, q, ti, td, wi, wd)
    # flat index: START comes from the build and there is no dense path
    fx = pdx.pdx_build(_dev(x))
    fs, ft = pdx.pdx_exact_tune(fx, _dev(q), 10, reps=1)
    timed = [(t["start_rows"], t["rounds"], t["dense_min"]) for t in ft if t["ms"] >= 0]
    assert timed == [(128, 2, 4), (128, 4, 4), (128, 8, 4)]
    assert fs["start_rows"] == 128 and fs["dense_min"] == 4
    # linear mode takes no tile path: only the defaults run
    ls, lt = pdx.pdx_exact_tune(fx, _dev(q), 10, mode="linear", reps=1)
    assert [t["ms"] >= 0 for t in lt].count(True) == 1 and ls == {"start_rows": 128, "rounds": 4, "dense_min": 4}
    for kw in (dict(rounds=65), dict(dense_min=34), dict(rounds=-1)):
        with pytest.raises(PdxError):
            pdx.pdx_search_exact(ix, _dev(q), 10, **kw)
