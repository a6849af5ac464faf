"""Comparison rules between the GPU results and the FP64 oracle.

Exact search (acceptance rule for float32 results): the returned ids must
be k distinct valid rows whose float64 distances, sorted, match the
oracle's k distances within a relative 1e-5 of the k-th distance (an id
outside the oracle's set is then a boundary tie), and every returned
float32 distance must equal its row's float64 distance within 1e-5
relative.  Integer-valued inputs make every distance exact, so there the
ids and distances must be identical.
"""
import numpy as np

from oracle.exact import sqdist

REL = 1e-5


def check_knn(x, q, got_ids, got_dist, want_ids, want_dist, rel=REL, exact=False):
    got_ids = np.asarray(got_ids)
    got_dist = np.asarray(got_dist, dtype=np.float64)
    nq, k = want_ids.shape
    assert got_ids.shape == (nq, k) and got_dist.shape == (nq, k)
    for i in range(nq):
        if exact:
            assert got_ids[i].tolist() == want_ids[i].tolist(), (i, got_ids[i], want_ids[i])
            assert np.array_equal(got_dist[i], want_dist[i]), (i, got_dist[i], want_dist[i])
            continue
        valid = want_ids[i] >= 0
        kv = int(valid.sum())
        gi = got_ids[i]
        assert np.all(gi[kv:] == -1) and np.all(np.isinf(got_dist[i, kv:])), (i, gi)
        g = gi[:kv]
        assert np.all(g >= 0) and np.all(g < x.shape[0]), (i, g)
        assert len(set(g.tolist())) == kv, (i, g)
        gamma = sqdist(x[g], q[i])
        dk = want_dist[i, kv - 1] if kv else 0.0
        tol = rel * dk + 1e-30
        assert np.all(np.abs(np.sort(gamma) - want_dist[i, :kv]) <= tol), (i, np.sort(gamma), want_dist[i, :kv])
        assert np.all(np.abs(got_dist[i, :kv] - gamma) <= rel * gamma + 1e-30), (i, got_dist[i, :kv], gamma)
        # reported order ascending
        assert np.all(np.diff(got_dist[i, :kv]) >= 0)


def check_knn_metric(x, q, got_ids, got_dist, want_ids, want_dist, metric, exact=False):
    """check_knn for the L1 and inner-product scores.  L1 keeps the relative
    1e-5 rule.  Inner-product scores (-q.v) are signed, and their float32
    rounding scales with |q| |v| rather than with the score: the tolerance
    is 1e-5 |q| max_v |v|."""
    from oracle.exact import METRICS
    score = METRICS[metric]
    got_ids = np.asarray(got_ids)
    got_dist = np.asarray(got_dist, dtype=np.float64)
    nq, k = want_ids.shape
    assert got_ids.shape == (nq, k) and got_dist.shape == (nq, k)
    xmax = float(np.sqrt((np.asarray(x, dtype=np.float64) ** 2).sum(1).max())) if x.shape[0] else 0.0
    for i in range(nq):
        if exact:
            assert got_ids[i].tolist() == want_ids[i].tolist(), (i, got_ids[i], want_ids[i])
            assert np.array_equal(got_dist[i], want_dist[i]), (i, got_dist[i], want_dist[i])
            continue
        valid = want_ids[i] >= 0
        kv = int(valid.sum())
        gi = got_ids[i]
        assert np.all(gi[kv:] == -1) and np.all(np.isinf(got_dist[i, kv:])), (i, gi)
        g = gi[:kv]
        assert np.all(g >= 0) and np.all(g < x.shape[0]), (i, g)
        assert len(set(g.tolist())) == kv, (i, g)
        gamma = score(x[g], q[i])
        if metric == "ip":
            tol = np.full(kv, REL * float(np.linalg.norm(np.asarray(q[i], dtype=np.float64))) * xmax + 1e-30)
            tk = tol
        else:
            dk = want_dist[i, kv - 1] if kv else 0.0
            tk = REL * dk + 1e-30
            tol = REL * gamma + 1e-30
        assert np.all(np.abs(np.sort(gamma) - want_dist[i, :kv]) <= tk), (i, np.sort(gamma), want_dist[i, :kv])
        assert np.all(np.abs(got_dist[i, :kv] - gamma) <= tol), (i, got_dist[i, :kv], gamma)
        assert np.all(np.diff(got_dist[i, :kv]) >= 0)
