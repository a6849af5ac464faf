"""Pins for the step-by-step PDXearch / PDX-BOND / ADSampling / IVF oracle.

* Hand-worked PDX-BOND runs (values computed, result) and orders.
* Invariant: PDX-BOND never changes the exact answer (Sections 2.3, 5:
  the partial distance is a lower bound), on integer inputs bit for bit
  and on real inputs, for every chunking and WARMUP/PRUNE threshold.
* ADSampling test: hand-worked thresholds; eps0 = inf reduces it to the
  exact bound, so the IVF search equals IVF-flat.
* IVF-flat with every bucket probed equals exact search.
"""
import numpy as np
import pytest

import synth
from oracle import exact, kmeans, mlp, pdxearch as px
from oracle.layout import column_means_f32
from tests.conftest import golden


def test_hand_bond_runs():
    g = golden("hand_bond.json")
    x = np.array(g["vectors"], dtype=np.float32)
    q = np.array(g["query"], dtype=np.float32)
    for c in g["cases"]:
        st = px.SearchStats()
        ids, dist = px.bond_search(x, q, c["k"], block=g["block"], chunk=g["chunk"], stats=st)
        assert ids.tolist() == c["ids"]
        assert dist.tolist() == c["dist"]
        assert st.values_computed == c["values_computed"]
        assert st.values_total == c["values_total"]


def test_hand_bond_orders():
    for c in golden("hand_bond.json")["order_cases"]:
        o = px.bond_order(np.array(c["query"], np.float32), np.array(c["means"], np.float32))
        assert o.tolist() == c["order"]


def test_hand_zone_orders():
    """Dimension zones worked by hand: zone scores and visit order."""
    for c in golden("hand_zones.json")["cases"]:
        qv = np.array(c["query"], np.float32)
        mu = np.array(c["means"], np.float32)
        z = c["zone"]
        nz = qv.size // z
        assert [float(np.abs(qv[i * z:(i + 1) * z] - mu[i * z:(i + 1) * z]).sum()) for i in range(nz)] == c["scores"]
        assert px.zone_order(qv, mu, z).tolist() == c["order"], c


@pytest.mark.parametrize("d", [1, 5, 31, 32, 96, 100, 960])
def test_zone_order_special_cases(d):
    """zone = 1 is the distance-to-means order (PDX-BOND's), zone = D the
    natural order; every order is a permutation made of whole zones in
    storage order, full zones by non-increasing summed key, a partial zone
    last."""
    rng = np.random.default_rng(d)
    qv = rng.standard_normal(d).astype(np.float32)
    mu = rng.standard_normal(d).astype(np.float32)
    qv[: d // 3] = mu[: d // 3]  # ties in the per-dimension key
    assert np.array_equal(px.zone_order(qv, mu, 1), px.bond_order(qv, mu))
    assert np.array_equal(px.zone_order(qv, mu, d), np.arange(d))
    key = np.abs(qv - mu).astype(np.float64)
    for z in (2, 7, 32):
        o = px.zone_order(qv, mu, z)
        assert np.array_equal(np.sort(o), np.arange(d))
        nz = d // z
        runs = o[: nz * z].reshape(nz, z)
        assert np.all(runs % z == np.arange(z)) and np.all(np.diff(runs, axis=1) == 1)
        sc = key[runs].sum(axis=1)
        assert np.all(np.diff(sc) <= 0)
        assert np.array_equal(o[nz * z:], np.arange(nz * z, d))


@pytest.mark.parametrize("zone", [None, 1, 7, 32])
def test_bond_ivf_search_equals_ivf_flat(zone):
    """PDX-BOND inside IVF, per-dimension or zone order, is exact within
    the probed buckets: integer inputs bit for bit, real inputs to 1e-12;
    pruning happens."""
    xi, qi = synth.integer_grid(2500, 64, 6, lo=-3, hi=3, seed=4)
    init = np.random.default_rng(4).choice(2500, 12, replace=False)
    c, lab, _ = kmeans.lloyd(xi, init, 3)
    lists = kmeans.lists_from_labels(lab, 12)
    mu = column_means_f32(xi)
    for i in range(qi.shape[0]):
        qq = qi[i].astype(np.float64)
        for nprobe in (1, 4, 12):
            fi, fd = px.ivf_flat(xi, lists, c, qq, 10, nprobe)
            bi, bd = px.bond_ivf_search(xi, lists, c, qq, 10, nprobe, mu, zone=zone)
            assert bi.tolist() == fi.tolist() and np.array_equal(bd, fd)
    x, q, c, lists = _small_ivf(seed=3, d=96)
    mu = column_means_f32(x)
    for i in range(q.shape[0]):
        qq = q[i].astype(np.float64)
        fi, fd = px.ivf_flat(x, lists, c, qq, 10, 6)
        st = px.SearchStats()
        bi, bd = px.bond_ivf_search(x, lists, c, qq, 10, 6, mu, zone=zone, stats=st)
        assert bi.tolist() == fi.tolist()
        np.testing.assert_allclose(bd, fd, rtol=1e-12)
        assert st.pruning_power > 0.1


def test_hand_ads_thresholds():
    g = golden("hand_ads.json")
    prune = px.make_ads_prunes(g["eps0"])
    for c in g["cases"]:
        got = bool(prune(np.array([c["partial"]]), g["tau"], c["d"], g["D"])[0])
        assert got == c["pruned"], c


@pytest.mark.parametrize("chunk", [1, 7, 32, 100])
@pytest.mark.parametrize("switch", [0.0, 0.2, 1.0])
def test_bond_equals_exact_integer(chunk, switch):
    x, q = synth.integer_grid(1200, 100, 4, lo=-3, hi=3, seed=11)
    want_i, want_d = exact.knn_exact(x, q, 10)
    for i in range(q.shape[0]):
        ids, dist = px.bond_search(x, q[i], 10, block=256, chunk=chunk, switch=switch)
        assert ids.tolist() == want_i[i].tolist()
        assert np.array_equal(dist, want_d[i])


def test_bond_equals_exact_real_and_prunes():
    x, q, _ = synth.workload("bond_1m_d960", n=6000, nq=3)
    want_i, want_d = exact.knn_exact(x, q, 10)
    for i in range(q.shape[0]):
        st = px.SearchStats()
        ids, dist = px.bond_search(x, q[i], 10, block=1000, chunk=32, stats=st)
        assert ids.tolist() == want_i[i].tolist()
        np.testing.assert_allclose(dist, want_d[i], rtol=1e-12)
        # on skewed data the bound must actually prune (Section 6.4)
        assert st.pruning_power > 0.3


def test_bond_small_first_block_and_k_over_n():
    x, q = synth.integer_grid(37, 5, 2, seed=5)
    want_i, want_d = exact.knn_exact(x, q, 50)
    for i in range(2):
        ids, dist = px.bond_search(x, q[i], 50, block=4, chunk=2)
        assert ids.tolist() == want_i[i].tolist()
        assert np.array_equal(dist, want_d[i])


def test_doubling_chunks_cover_once():
    ch = px.doubling_chunks(np.arange(100))
    assert [c.size for c in ch] == [2, 4, 8, 16, 32, 38]
    assert np.array_equal(np.concatenate(ch), np.arange(100))
    assert px.ads_delta_d(960) == 32 and px.ads_delta_d(64) == 16


def _small_ivf(seed=1, n=3000, d=64, nlist=24):
    mix = synth.anisotropic_unit_mixture(d, 16, seed)
    x = mix.data(n)
    q = mix.queries(6)
    init = np.random.default_rng(seed).choice(n, nlist, replace=False)
    c, lab, _ = kmeans.lloyd(x, init, 5)
    return x, q, c, kmeans.lists_from_labels(lab, nlist)


def test_ivf_flat_all_buckets_is_exact():
    x, q, c, lists = _small_ivf()
    want_i, want_d = exact.knn_exact(x, q, 10)
    for i in range(q.shape[0]):
        ids, dist = px.ivf_flat(x, lists, c, q[i].astype(np.float64), 10, len(lists))
        assert ids.tolist() == want_i[i].tolist()
        np.testing.assert_allclose(dist, want_d[i], rtol=1e-12)


def test_ads_eps_inf_equals_ivf_flat_and_recall_monotone():
    x, q, c, lists = _small_ivf()
    truth, _ = exact.knn_exact(x, q, 10)
    prev = -1.0
    for nprobe in (1, 3, 6, 24):
        got_flat, got_ads, got_inf = [], [], []
        for i in range(q.shape[0]):
            qq = q[i].astype(np.float64)
            fi, fd = px.ivf_flat(x, lists, c, qq, 10, nprobe)
            ii, idd = px.ads_ivf_search(x, lists, c, qq, 10, nprobe, eps0=np.inf)
            assert ii.tolist() == fi.tolist()
            np.testing.assert_allclose(idd, fd, rtol=1e-12)
            ai, _ = px.ads_ivf_search(x, lists, c, qq, 10, nprobe, eps0=2.1)
            got_flat.append(fi)
            got_ads.append(ai)
        r_flat = exact.recall_at_k(truth, np.stack(got_flat))
        r_ads = exact.recall_at_k(np.stack(got_flat), np.stack(got_ads))
        assert r_flat >= prev
        prev = r_flat
        assert r_ads >= 0.9
    assert prev == 1.0


def test_probe_order_ties_by_bucket_id():
    c = np.array([[1.0, 0], [0, 1.0], [-1.0, 0], [3.0, 0]])
    order = px.ivf_probe_order(c, np.zeros(2), 3)
    assert order.tolist() == [0, 1, 2]


def test_means_rounding_is_single():
    x = np.array([[1.0, 0.1], [2.0, 0.2], [4.0, 0.3]], dtype=np.float32)
    m = column_means_f32(x)
    assert m[0] == np.float32(7.0 / 3.0)
    assert m[1] == np.float32((np.float64(np.float32(0.1)) + np.float64(np.float32(0.2)) + np.float64(np.float32(0.3))) / 3)


# ---------------------------------------------------------------------------
# the learned prune multiplier's search (one multiplier per bucket and test)
# ---------------------------------------------------------------------------

def _ads_rows(eps0, d, dd, nprobe):
    pts = np.arange(dd, d, dd, dtype=np.float64)
    return np.tile((1.0 + eps0 / np.sqrt(pts)) ** 2, (nprobe - 1, 1))


def test_table_search_reduces_to_ads_and_to_ivf_flat():
    x, q, c, lists = _small_ivf(seed=4)
    nprobe, dd = 8, 16
    for i in range(q.shape[0]):
        qq = q[i].astype(np.float64)
        ai, ad = px.ads_ivf_search(x, lists, c, qq, 10, nprobe, eps0=2.1, delta_d=dd)
        ti, td = px.learned_ivf_search(x, lists, c, qq, 10, nprobe, _ads_rows(2.1, 64, dd, nprobe), dd)
        assert ti.tolist() == ai.tolist() and np.array_equal(td, ad)
        fi, fd = px.ivf_flat(x, lists, c, qq, 10, nprobe)
        ti, td = px.learned_ivf_search(x, lists, c, qq, 10, nprobe, np.full((nprobe - 1, 3), 1e30), dd)
        assert ti.tolist() == fi.tolist()
        # multipliers of 0 drop every vector with a positive partial: only START remains
        si, sd = px.ivf_flat(x, lists, c, qq, 10, 1)
        ti, td = px.learned_ivf_search(x, lists, c, qq, 10, nprobe, np.zeros((nprobe - 1, 3)), dd)
        assert ti.tolist() == si.tolist()


def test_bounds_from_the_targets_keep_every_neighbour():
    """Each bucket's bound at the largest target of its returned neighbours
    (none: multiplier 0) keeps every neighbour, because the threshold in
    force never falls below the final k-th distance: the search returns
    IVF-flat's result, while the same multipliers halved lose one."""
    x, q, c, lists = _small_ivf(seed=5, n=4000, d=64, nlist=20)
    nprobe, dd, k = 10, 16, 10
    pts = mlp.test_points(64, dd)
    labels = np.empty(x.shape[0], np.int64)
    for l, rows in enumerate(lists):
        labels[rows] = l
    lost = 0
    for i in range(q.shape[0]):
        qq = q[i].astype(np.float64)
        fi, fd = px.ivf_flat(x, lists, c, qq, k, nprobe)
        probe = px.ivf_probe_order(c, qq, nprobe)
        rank = {int(b): r for r, b in enumerate(probe)}
        t = mlp.prune_targets(x, qq, fi, fd[-1], dd)
        eps = np.full(nprobe - 1, -np.inf)
        for a, v in enumerate(fi):
            r = rank[int(labels[v])]
            if r >= 1:
                eps[r - 1] = max(eps[r - 1], t[a])
        mult = np.array([[0.0 if e == -np.inf else mlp.multiplier(e, c1) * (1 + 1e-12) for c1 in pts]
                         for e in eps])
        gi, gd = px.learned_ivf_search(x, lists, c, qq, k, nprobe, mult, dd)
        assert gi.tolist() == fi.tolist()
        if mult.max() > 0:
            gi2, _ = px.learned_ivf_search(x, lists, c, qq, k, nprobe, mult * 0.5, dd)
            lost += gi2.tolist() != fi.tolist()
    assert lost >= 1


def test_bsa_hand_worked():
    """BSA's Cauchy-Schwarz test (Section 2.3; reading in oracle.pdxearch),
    thresholds worked by hand (tests/golden/hand_bsa.json)."""
    g = golden("hand_bsa.json")
    q = np.array(g["query"])
    for c in g["cases"]:
        x = np.array([c["x"]])
        partial = np.array([c["partial"]])
        got = px.make_bsa_prunes(x, q, c["m"])(partial, g["tau"], g["dims_seen"], g["D"])
        assert bool(got[0]) == c["pruned"], c
        # at d = D the test is exact whatever m
        full = float(((x[0] - q) ** 2).sum())
        assert bool(px.make_bsa_prunes(x, q, c["m"])(np.array([full]), g["tau"], g["D"], g["D"])[0]) == (full > g["tau"])


def test_bsa_with_m_one_is_exact_within_buckets():
    """With m = 1 the estimate is a lower bound (Cauchy-Schwarz), so the
    search equals IVF-flat while pruning; a planted sign error in the cross
    term loses neighbours."""
    rng = np.random.default_rng(21)
    n, d, nlist, k = 3000, 64, 8, 10
    x = (rng.standard_normal((n, d)) * np.linspace(2.0, 0.3, d)[None, :])
    q = rng.standard_normal((12, d)) * np.linspace(2.0, 0.3, d)[None, :]
    cen, assign, _ = kmeans.lloyd(x, rng.choice(n, nlist, replace=False), 5)
    lists = [np.flatnonzero(assign == l) for l in range(nlist)]
    st = px.SearchStats()
    lost_planted = 0
    for qq in q:
        want = px.ivf_flat(x, lists, cen, qq, k, 4)
        got = px.bsa_ivf_search(x, lists, cen, qq, k, 4, 1.0, delta_d=16, stats=st)
        assert got[0].tolist() == want[0].tolist()
        np.testing.assert_allclose(got[1], want[1], rtol=1e-12)

        def planted(xb, qv, m):
            xb, qv = np.asarray(xb, np.float64), np.asarray(qv, np.float64)

            def prune(partial, tau, seen, dd):
                if seen >= dd:
                    return partial > tau
                xr = np.sqrt((xb[:, seen:] ** 2).sum(axis=1))
                qr = float(np.sqrt((qv[seen:] ** 2).sum()))
                return partial + qr * qr + xr * xr + 2.0 * m * qr * xr > tau
            return prune
        probe = px.ivf_probe_order(cen, qq, 4)
        blocks = [lists[p] for p in probe]
        bad = px.pdxearch(x, qq, k, blocks, px.fixed_chunks(np.arange(d), 16), [planted(x[b], qq, 1.0) for b in blocks])
        lost_planted += len(set(want[0].tolist()) - set(bad[0].tolist()))
    assert st.pruning_power > 0.05   # the bound prunes
    assert lost_planted > 0          # the pin catches a sign error
