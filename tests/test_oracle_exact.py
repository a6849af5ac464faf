"""Pins for the exact-KNN oracle (Section 2.1).  CPU only.

Each pin comes from outside the oracle: hand-worked values, scipy's
pairwise-distance routine with a full sort, exact integer arithmetic,
and special cases (query equal to a row, duplicates, k > n).
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import synth
from oracle import exact
from tests.conftest import golden


def _full_sort_topk(x, q, k):
    """scipy cdist + a complete lexicographic sort of every (dist, id)."""
    d = cdist(np.atleast_2d(q).astype(np.float64), x.astype(np.float64), "sqeuclidean")[0]
    ids = np.arange(x.shape[0])
    o = np.lexsort((ids, d))
    return ids[o][:k], d[o][:k]


def test_hand_worked_cases():
    g = golden("hand_knn.json")
    x = np.array(g["vectors"], dtype=np.float32)
    for c in g["cases"]:
        ids, dist = exact.knn_exact(x, np.array([c["query"]], dtype=np.float32), c["k"])
        want_d = np.array([np.inf if v == "inf" else v for v in c["dist"]], dtype=np.float64)
        assert ids[0].tolist() == c["ids"]
        assert np.array_equal(dist[0], want_d)


@pytest.mark.parametrize("n,d,k", [(1, 1, 1), (7, 3, 3), (200, 17, 10), (1500, 65, 32)])
def test_matches_scipy_full_sort(n, d, k):
    rng = np.random.default_rng(n * 31 + d)
    x = rng.standard_normal((n, d)).astype(np.float32)
    q = rng.standard_normal((4, d)).astype(np.float32)
    ids, dist = exact.knn_exact(x, q, k)
    for i in range(q.shape[0]):
        wi, wd = _full_sort_topk(x, q[i], k)
        kk = min(k, n)
        assert ids[i, :kk].tolist() == wi.tolist()
        np.testing.assert_allclose(dist[i, :kk], wd, rtol=1e-12, atol=0)


def test_integer_inputs_exact_and_c_matches_numpy(oracle_c):
    x, q = synth.integer_grid(3000, 100, 8)
    ids, dist = exact.knn_exact(x, q, 20)
    ci, cd = oracle_c.knn_exact_c(x, q, 20, threads=2)
    assert np.array_equal(ids, ci)
    assert np.array_equal(dist, cd)
    # integer distances: exact integers, heavy ties broken by id
    assert np.all(dist == np.round(dist))
    for i in range(q.shape[0]):
        wi, wd = _full_sort_topk(x, q[i], 20)
        assert ids[i].tolist() == wi.tolist()


def test_c_matches_numpy_real_values(oracle_c):
    x, q, _ = synth.workload("linear_10k_d128", n=2000, nq=5)
    ids, dist = exact.knn_exact(x, q, 10)
    ci, cd = oracle_c.knn_exact_c(x, q, 10)
    assert np.array_equal(ids, ci)
    np.testing.assert_allclose(cd, dist, rtol=1e-12)


def test_query_equal_to_row_and_duplicates(oracle_c):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((50, 9)).astype(np.float32)
    x[30] = x[12]  # duplicate row
    q = x[12:13].copy()
    for fn in (exact.knn_exact, lambda a, b, k: oracle_c.knn_exact_c(a, b, k)):
        ids, dist = fn(x, q, 3)
        assert ids[0, :2].tolist() == [12, 30]
        assert dist[0, 0] == 0.0 and dist[0, 1] == 0.0
        assert dist[0, 2] > 0


def test_k_larger_than_n_pads(oracle_c):
    x = np.arange(6, dtype=np.float32).reshape(3, 2)
    ids, dist = oracle_c.knn_exact_c(x, x[:1], 5)
    assert ids[0].tolist() == [0, 1, 2, -1, -1]
    assert np.isinf(dist[0, 3:]).all()


def test_recall_definition():
    t = np.array([[1, 2, 3, 4]])
    assert exact.recall_at_k(t, np.array([[4, 3, 9, 8]])) == 0.5
    assert exact.recall_at_k(t, t) == 1.0


# ---------------------------------------------------------------------------
# L1 and inner product (the other two kernels of Section 3's listing)
# ---------------------------------------------------------------------------

def test_metrics_hand_worked():
    # rows (0,0), (1,2), (3,-1), (-2,2); query (1,1)
    x = np.array([[0.0, 0.0], [1.0, 2.0], [3.0, -1.0], [-2.0, 2.0]])
    q = np.array([[1.0, 1.0]])
    # L1: 2, 1, 4, 4 -> ids 1, 0, then the tie 2 / 3 by id
    i, d = exact.knn_exact(x, q, 4, metric="l1")
    assert i[0].tolist() == [1, 0, 2, 3] and d[0].tolist() == [1.0, 2.0, 4.0, 4.0]
    # inner products 0, 3, 2, 0 -> scores -3, -2, then 0, 0 by id
    i, d = exact.knn_exact(x, q, 4, metric="ip")
    assert i[0].tolist() == [1, 2, 0, 3] and d[0].tolist() == [-3.0, -2.0, 0.0, 0.0]


def test_l1_matches_scipy_cityblock():
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(21)
    x = rng.standard_normal((300, 17)).astype(np.float32)
    q = rng.standard_normal((5, 17)).astype(np.float32)
    i, d = exact.knn_exact(x, q, 12, metric="l1")
    ref = cdist(q.astype(np.float64), x.astype(np.float64), "cityblock")
    for r in range(5):
        o = np.lexsort((np.arange(300), ref[r]))[:12]
        assert i[r].tolist() == o.tolist()
        np.testing.assert_allclose(d[r], ref[r][o], rtol=1e-13)


def test_inner_product_brute_force_and_unit_norm_equivalence():
    rng = np.random.default_rng(22)
    x = rng.standard_normal((40, 6))
    q = rng.standard_normal((3, 6))
    i, d = exact.knn_exact(x, q, 7, metric="ip")
    for r in range(3):
        ip = [sum(x[v, j] * q[r, j] for j in range(6)) for v in range(40)]
        o = sorted(range(40), key=lambda v: (-ip[v], v))[:7]
        assert i[r].tolist() == o
        np.testing.assert_allclose(d[r], [-ip[v] for v in o], rtol=1e-12)
    # on unit vectors |q - v|^2 = 2 - 2 q.v: the same order as L2
    xn = x / np.linalg.norm(x, axis=1, keepdims=True)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    i2, d2 = exact.knn_exact(xn, qn, 7)
    ii, di = exact.knn_exact(xn, qn, 7, metric="ip")
    assert np.array_equal(i2, ii)
    np.testing.assert_allclose(d2, 2.0 + 2.0 * di, rtol=1e-12, atol=1e-12)


def test_blocked_brute_force_equals_plain():
    rng = np.random.default_rng(23)
    x = rng.standard_normal((1000, 9)).astype(np.float32)
    q = rng.standard_normal((4, 9)).astype(np.float32)
    for metric in ("l2", "l1", "ip"):
        for k in (1, 10, 1200):
            a = exact.knn_exact(x, q, k, metric=metric)
            b = exact.knn_exact_blocked(x, q, k, metric=metric, block=97)
            assert np.array_equal(a[0], b[0]) and np.allclose(a[1], b[1], rtol=1e-13, atol=0)
