"""GPU visit orders and pruning counts against the oracle, through the C ABI.

* Section 5 (PDX-BOND, distance to means; dimension zones, Figure "dz"):
  the order every query's search visits its dimensions in, read through
  pdx_query_order (the searches' own query preparation), equals
  oracle.pdxearch.bond_order / zone_order element by element, including the
  16-bit LDS tile offsets the exact search's tile scan reads.  Inputs make
  the means exact on both sides (dyadic values over a power-of-two row
  count), so the float32 keys are identical and every tie must go by
  dimension (or zone) index.  D = 37 (a short last zone) and D = 960.
* Section 2.3 (pruning power) and Section 4: with the exact top-k inside the
  START block, the threshold is fixed for the whole pruned scan, so the
  (query, vector) pairs surviving each chunk are determined by the data;
  the GPU's per-chunk survivor counts and its count of evaluated values
  equal oracle.pdxearch.SearchStats of the same search bit for bit
  (integer inputs, every partial exact), on the LDS-tile path (D = 128)
  and on the vectorgroup path (D = 100, a short last chunk).
"""
import numpy as np
import pytest

from oracle import exact, pdxearch as px
from oracle.layout import column_means_f32
from oracle.rotation import orthogonal_from_gaussian, rotate_rows

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


def _orders(pdx, ix, q, order):
    import torch
    perm, qval, off = pdx.pdx_query_order(ix, _dev(q), order, tile_offsets=ix.d * 32 < 65536)
    torch.cuda.synchronize()
    off = None if off is None else off.cpu().numpy().view(np.uint16)
    return perm.cpu().numpy(), qval.cpu().numpy(), off


def _exact_mean_rows(rng, n, d, dyadic):
    """Rows whose column means are exact in float32 on any summation order:
    each column is c_j plus values and their negatives (n even, a power of
    two), so the mean is c_j itself."""
    half = n // 2
    if dyadic:
        c = rng.integers(-2048, 2048, d) / 1024.0
        r = rng.integers(-4096, 4096, (half, d)) / 1024.0
    else:
        c = rng.integers(-3, 4, d).astype(np.float64)
        r = rng.integers(-5, 6, (half, d)).astype(np.float64)
    x = np.concatenate([c + r, c - r]).astype(np.float32)
    return x[rng.permutation(n)], c.astype(np.float32)


def _queries(rng, c, nq):
    """Gaussian queries (the first nq rows), dyadic ones, integer offsets
    from the means (ties in |q_j - mean_j|), the means themselves (every key
    0: ties everywhere) and zone-constant offsets (tied zone scores).  A
    zone's score is a float32 sum on the GPU and a float64 sum in the
    oracle; on every query but the Gaussian ones both sums are exact."""
    d = c.size
    real = (c + rng.standard_normal((nq, d))).astype(np.float32)
    dy = (c + rng.integers(-4096, 4097, (nq, d)) / 1024.0).astype(np.float32)
    ints = (c + rng.integers(-3, 4, (nq, d))).astype(np.float32)
    zoned = np.repeat(rng.integers(0, 3, (nq, (d + 31) // 32)), 32, axis=1)[:, :d]
    zq = (c + zoned).astype(np.float32)
    return np.concatenate([real, dy, ints, c[None, :], zq]), nq


@pytest.mark.parametrize("d", [37, 960])
def test_flat_orders_equal_oracle(pdx, d):
    rng = np.random.default_rng(d)
    x, c = _exact_mean_rows(rng, 4096, d, dyadic=True)
    mu = column_means_f32(x)
    assert np.array_equal(mu, c)  # the premise: exact means
    q, ng = _queries(rng, c, 6)
    print(f"flat orders d={d} nq={q.shape[0]}", flush=True)
    ix = pdx.pdx_build(_dev(x))
    for name, ref in (("bond", lambda qq: px.bond_order(qq, mu)), ("zones", lambda qq: px.zone_order(qq, mu, 32)),
                      ("natural", lambda qq: np.arange(d))):
        perm, qval, off = _orders(pdx, ix, q, name)
        for i in range(ng if name == "zones" else 0, q.shape[0]):
            want = ref(q[i])
            assert perm[i].tolist() == want.tolist(), (name, i)
            assert np.array_equal(qval[i], q[i][want]), (name, i)
            assert off[i].tolist() == (32 * want).tolist(), (name, i)


def test_bucket_layout_orders_equal_oracle(pdx):
    """An IVF index without rotation: the means are those of the stored rows
    (the same rows in bucket order)."""
    rng = np.random.default_rng(5)
    d = 96
    x, c = _exact_mean_rows(rng, 2048, d, dyadic=False)
    q, ng = _queries(rng, c, 8)
    init = rng.choice(x.shape[0], 12, replace=False).astype(np.int64)
    print("bucket-layout orders", flush=True)
    ix = pdx.pdx_ivf_build(_dev(x), 12, None, _dev(init), kmeans_iters=3)
    mu = column_means_f32(x)
    for name, ref in (("bond", lambda qq: px.bond_order(qq, mu)), ("zones", lambda qq: px.zone_order(qq, mu, 32))):
        perm, qval, off = _orders(pdx, ix, q, name)
        for i in range(ng if name == "zones" else 0, q.shape[0]):
            want = ref(q[i])
            assert perm[i].tolist() == want.tolist(), (name, i)
            assert off[i].tolist() == (32 * want).tolist(), (name, i)


def test_rotated_index_order_is_a_valid_bond_order(pdx):
    """A rotated index rotates the query on the matrix cores, so near-equal
    keys may fall either way; the order must be a permutation whose oracle
    keys (FP64 rotation of the same Gaussian) never increase by more than
    the rounding of the rotated values."""
    rng = np.random.default_rng(7)
    n, d, nlist = 3000, 64, 10
    x = rng.standard_normal((n, d)).astype(np.float32)
    q = rng.standard_normal((5, d)).astype(np.float32)
    g = rng.standard_normal((d, d))
    init = rng.choice(n, nlist, replace=False).astype(np.int64)
    print("rotated order", flush=True)
    ix = pdx.pdx_ivf_build(_dev(x), nlist, _dev(g), _dev(init), kmeans_iters=2)
    rot = orthogonal_from_gaussian(g)
    mu = rotate_rows(x.astype(np.float64), rot).mean(axis=0)
    perm, qval, _ = _orders(pdx, ix, q, "bond")
    qr = rotate_rows(q.astype(np.float64), rot)
    for i in range(q.shape[0]):
        assert sorted(perm[i].tolist()) == list(range(d))
        key = np.abs(qr[i] - mu)[perm[i]]
        assert np.all(np.diff(key) <= 1e-4 * (1.0 + key.max())), i
        np.testing.assert_allclose(qval[i], qr[i][perm[i]], rtol=0, atol=1e-4)


def _stats_workload(d, seed):
    """Integer rows: a START block of near neighbours of every query (noise
    in {-1, 0, 1}) and a later block with rows near each query (noise
    {-1, 0, 1} with 0 rarer, so their partial distances cross the
    threshold after a few chunks) and far rows."""
    rng = np.random.default_rng(seed)
    nq, n_start, n_rest = 24, 2048, 64 * 160
    cen = rng.integers(-4, 5, (nq, d))
    own_s = np.arange(n_start) % nq
    xs = cen[own_s] + rng.integers(-1, 2, (n_start, d))
    own_r = rng.integers(0, nq, n_rest)
    noise = rng.choice([-1, 0, 1], size=(n_rest, d), p=[0.4, 0.2, 0.4])
    xr = cen[own_r] + noise
    x = np.concatenate([xs, xr]).astype(np.float32)
    return x, cen.astype(np.float32), n_start


@pytest.mark.parametrize("d", [128, 100])
def test_survivors_per_chunk_equal_oracle(pdx, d):
    import torch
    k = 10
    x, q, n_start = _stats_workload(d, 11 + d)
    mu = column_means_f32(x)
    blocks = [np.arange(n_start), np.arange(n_start, x.shape[0])]
    nch = (d + 31) // 32
    want_surv = np.zeros(nch, np.int64)
    want_vals = 0
    for i in range(q.shape[0]):
        # the premise: START holds the exact top-k, so the threshold is fixed
        st_start = px.SearchStats()
        px.pdxearch(x, q[i], k, blocks[:1], px.fixed_chunks(px.bond_order(q[i], mu), 32), px.bond_prunes, 2.0,
                    st_start)
        wi, wd = exact.knn_exact(x, q[i][None], k)
        assert np.all(wi[0] < n_start), i
        st = px.SearchStats()
        ids, dist = px.pdxearch(x, q[i], k, blocks, px.fixed_chunks(px.bond_order(q[i], mu), 32), px.bond_prunes,
                                2.0, st)  # switch above 1: PRUNE after the first chunk, as on the GPU
        assert ids.tolist() == wi[0].tolist()
        s = np.array(st.survivors_per_chunk, np.int64)
        want_surv[:s.size] += s
        want_vals += st.values_computed - n_start * d
    assert np.count_nonzero(want_surv) >= 2  # survivors spread over several chunks
    print(f"survivors per chunk d={d}: oracle {want_surv.tolist()}", flush=True)
    ix = pdx.pdx_build(_dev(x), start_rows=n_start)
    surv = torch.zeros(nch, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    ids, dist = pdx.pdx_search_exact(ix, _dev(q), k, mode="bond", counters=cnt, chunk_survivors=surv)
    torch.cuda.synchronize()
    wi, wd = exact.knn_exact(x, q, k)
    assert np.array_equal(ids.cpu().numpy(), wi)
    assert np.array_equal(dist.cpu().numpy().astype(np.float64), wd)
    got = surv.cpu().numpy()
    assert got.tolist() == want_surv.tolist()
    c = cnt.cpu().numpy()
    assert int(c[0]) == q.shape[0] * n_start * d  # START: every value of its block
    assert int(c[2]) == want_vals  # pruned scan: the values the oracle computed
    # the plain search (no instrumentation) returns the same bits
    ids2, dist2 = pdx.pdx_search_exact(ix, _dev(q), k, mode="bond")
    torch.cuda.synchronize()
    assert np.array_equal(ids2.cpu().numpy(), wi)
