"""pdx_search_exact_noalloc (static device scratch, no allocation) against
pdx_search_exact (caller workspace) through the C ABI: the same kernels, so
the same bits; both checked against the FP64 oracle under the tie rule.
Two calls in a row, the second with fewer queries (the scratch keeps the
first call's contents), on a flat index and on a bucket layout; a request
beyond the scratch is refused with PDX_EWORKSPACE."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import exact
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


def _noalloc(pdx, ix, q, k, mode="bond"):
    import torch
    from paper_2503_04422_amd import _lib
    nq = q.shape[0]
    p = _lib.pdx_search_params(pdx.api._MODES[mode], 0, 0, 0, None, None, _lib.PDX_METRIC_L2, 0, None)
    ids = torch.full((nq, k), -7, dtype=torch.int64, device=q.device)
    dist = torch.full((nq, k), -7.0, dtype=torch.float32, device=q.device)
    st = _lib.lib.pdx_search_exact_noalloc(ix.handle, q.data_ptr(), nq, k, ctypes.byref(p), ids.data_ptr(),
                                           dist.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return st, ids, dist


def _both(pdx, ix, x, q_np, k, mode):
    import torch
    from paper_2503_04422_amd import _lib
    q = _dev(q_np)
    st, ids, dist = _noalloc(pdx, ix, q, k, mode)
    assert st == _lib.PDX_OK, _lib.lib.pdx_last_error()
    wi, wd = pdx.pdx_search_exact(ix, q, k, mode=mode)
    torch.cuda.synchronize()
    gi, gd = ids.cpu().numpy(), dist.cpu().numpy()
    assert np.array_equal(gi, wi.cpu().numpy())
    assert np.array_equal(gd.view(np.int32), wd.cpu().numpy().view(np.int32))
    oi, od = exact.knn_exact_c(x, q_np, k)
    check_knn(x, q_np, gi, gd, oi, od)


@pytest.mark.parametrize("layout", ["flat", "buckets"])
def test_noalloc_equals_workspace_search(pdx, layout):
    x, q, _ = synth.workload("bond_1m_d960", n=20_000, nq=48)
    print(f"noalloc layout={layout}", flush=True)
    if layout == "flat":
        ix = pdx.pdx_build(_dev(x), start_rows=4096)
    else:
        rng = np.random.default_rng(3)
        init = rng.choice(x.shape[0], 40, replace=False).astype(np.int64)
        ix = pdx.pdx_ivf_build(_dev(x), 40, None, _dev(init), kmeans_iters=4)
    _both(pdx, ix, x, q, 10, "bond")          # first call
    _both(pdx, ix, x, q[:7], 5, "bond")       # second, smaller: stale scratch from the first
    _both(pdx, ix, x, q[:20], 10, "linear")


def test_noalloc_refuses_beyond_scratch(pdx):
    import torch
    from paper_2503_04422_amd import _lib
    x, q, _ = synth.workload("bond_1m_d960", n=20_000, nq=8)
    ix = pdx.pdx_build(_dev(x), start_rows=4096)
    big = 4096
    need = pdx.pdx_search_exact_workspace(ix, big, 64)
    assert need > _lib.PDX_NOALLOC_SCRATCH_BYTES
    qb = torch.zeros((big, x.shape[1]), dtype=torch.float32, device="cuda")
    st, ids, _ = _noalloc(pdx, ix, qb, 64)
    assert st == _lib.PDX_EWORKSPACE
    assert b"scratch" in _lib.lib.pdx_last_error()
    torch.cuda.synchronize()
    assert int(ids[0, 0]) == -7  # nothing was enqueued
