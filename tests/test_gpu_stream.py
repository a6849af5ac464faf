"""Searches on a side stream while torch's current stream allocates and
frees: the binding makes the call's own temporaries (workspace, outputs,
contiguous copies) on the stream the library's kernels run on, so the
caching allocator cannot hand their memory to the other stream's work
while the kernels still read it.  Results must equal the same search on
the current stream, and the oracle."""
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


def test_side_stream_search_with_busy_current_stream(pdx):
    import torch
    x, q, _ = synth.workload("bond_1m_d960", n=30_000, nq=64)
    xd = torch.from_numpy(x).cuda()
    ix = pdx.pdx_build(xd, start_rows=4096)
    # a non-contiguous query view forces a copy inside the call
    qd = torch.from_numpy(np.ascontiguousarray(q.T)).cuda().t()
    ref_i, ref_d = pdx.pdx_search_exact(ix, qd.contiguous(), 10)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    outs = []
    for rep in range(4):
        ids, dist = pdx.pdx_search_exact(ix, qd, 10, stream=side)
        outs.append((ids, dist))
        # the current stream churns through allocations of the same sizes
        for _ in range(8):
            junk = torch.full((64 * 1024 * 1024 // 4,), float(rep), device="cuda")
            junk.mul_(2.0)
            del junk
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for ids, dist in outs:
        assert torch.equal(ids, ref_i)
        assert torch.equal(dist, ref_d)
    oi, od = exact.knn_exact_c(x, q, 10)
    check_knn(x, q, ref_i.cpu().numpy(), ref_d.cpu().numpy(), oi, od)
