"""GPU parity of the distance kernels without a search (the kernel study of
Section 6.4; Section 3's layout and listing) against the FP64 oracle,
through the C ABI.

* pdx_layout_blocks equals the oracle's PDX layout bit for bit for every
  block size, ragged n and D;
* integer inputs: every score is exact, so both layouts equal the oracle
  bit for bit, every metric and block size;
* N(0, 1) inputs: within the chunked-sum bound (34 + D/32) 2^-24 of the
  sum of |terms| (positive terms for L2 and L1, |q_j v_j| for the inner
  product), and the PDX and row-major layouts return the same bits, with
  one segment (D <= 32) and with several (the dimensions split over the
  waves of a workgroup);
* the largest collection of the study's grid (131,072 vectors) at D =
  2048, sampled against the oracle; nq = 0 and a batch of queries.
"""
import numpy as np
import pytest

import synth
from oracle import exact
from oracle.layout import to_pdx

pytestmark = pytest.mark.gpu

BLOCKS = (16, 32, 64, 128, 256, 512)
SCORES = {"l2": exact.sqdist, "l1": exact.l1dist, "ip": exact.neg_ip}


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


def _want(x, q, metric):
    return np.stack([SCORES[metric](x, qi) for qi in q])


def _abs_terms(x, q, metric):
    x64, q64 = np.asarray(x, np.float64), np.asarray(q, np.float64)
    if metric == "ip":
        return np.abs(q64) @ np.abs(x64).T
    return np.stack([SCORES[metric](x, qi) for qi in q])


@pytest.mark.parametrize("n,d", [(1000, 37), (64, 8), (5, 3), (700, 130)])
def test_layout_blocks_equals_oracle(pdx, n, d):
    x, _ = synth.standard_normal(n, d, 1, seed=n + d)
    for b in BLOCKS:
        print(f"layout n={n} d={d} block={b}", flush=True)
        got = _np(pdx.pdx_layout_blocks(_dev(x), b))
        assert np.array_equal(got, to_pdx(x, b)), b


@pytest.mark.parametrize("n,d", [(1000, 37), (777, 128), (64, 8), (3, 1)])
def test_integer_inputs_bit_exact(pdx, n, d):
    x, q = synth.integer_grid(n, d, 3, lo=-5, hi=5, seed=n * 3 + d)
    xd, qd = _dev(x), _dev(q)
    for metric in ("l2", "l1", "ip"):
        want = _want(x, q, metric)
        print(f"integer n={n} d={d} {metric} nary", flush=True)
        got = _np(pdx.pdx_distances(xd, qd, layout="nary", metric=metric))
        assert np.array_equal(got.astype(np.float64), want)
        for b in BLOCKS:
            print(f"integer n={n} d={d} {metric} block={b}", flush=True)
            blocks = pdx.pdx_layout_blocks(xd, b)
            got = _np(pdx.pdx_distances(blocks, qd, n=n, layout="pdx", metric=metric))
            assert np.array_equal(got.astype(np.float64), want), b


@pytest.mark.parametrize("n,d", [(3000, 8), (1500, 100), (2049, 768), (300, 8192)])
def test_normal_inputs_within_bound_and_layouts_agree(pdx, n, d):
    x, q = synth.standard_normal(n, d, 2, seed=d)
    xd, qd = _dev(x), _dev(q)
    bound = (34 + (d + 31) // 32) * 2.0 ** -24
    for metric in ("l2", "l1", "ip"):
        want = _want(x, q, metric)
        tol = bound * _abs_terms(x, q, metric) + 1e-30
        print(f"normal n={n} d={d} {metric} nary", flush=True)
        ref = _np(pdx.pdx_distances(xd, qd, layout="nary", metric=metric))
        assert np.all(np.abs(ref.astype(np.float64) - want) <= tol)
        for b in BLOCKS:
            print(f"normal n={n} d={d} {metric} block={b}", flush=True)
            got = _np(pdx.pdx_distances(pdx.pdx_layout_blocks(xd, b), qd, n=n, layout="pdx", metric=metric))
            assert np.array_equal(got, ref), b


def test_largest_collection_sampled_and_edges(pdx):
    import torch
    n, d = synth.KERNEL_STUDY_N[-1], 2048
    x, q = synth.standard_normal(n, d, 1)
    print(f"largest n={n} d={d}", flush=True)
    xd, qd = _dev(x), _dev(q)
    ref = _np(pdx.pdx_distances(xd, qd, layout="nary"))
    got = _np(pdx.pdx_distances(pdx.pdx_layout_blocks(xd, 64), qd, n=n, layout="pdx"))
    assert np.array_equal(got, ref)
    sample = np.random.default_rng(1).choice(n, 64, replace=False)
    sample[0], sample[1] = 0, n - 1
    want = exact.sqdist(x[sample], q[0])
    bound = (34 + d // 32) * 2.0 ** -24
    assert np.all(np.abs(got[0, sample].astype(np.float64) - want) <= bound * want)
    # no queries; fewer vectors than one block
    empty = pdx.pdx_distances(xd[:10], torch.empty((0, d), device="cuda"), layout="nary")
    assert empty.shape == (0, 10)
    # (the segment count follows n, so compare layouts at the same n)
    small = _np(pdx.pdx_distances(pdx.pdx_layout_blocks(xd[:10], 512), qd, n=10, layout="pdx"))
    assert np.array_equal(small, _np(pdx.pdx_distances(xd[:10], qd, layout="nary")))
    want = exact.sqdist(x[:10], q[0])
    assert np.all(np.abs(small[0].astype(np.float64) - want) <= bound * want)
