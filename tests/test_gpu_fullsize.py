"""Full-size parity of the IVF search on the two large workloads, sampled
against the FP64 oracle (the oracle cannot run k-means at this size, and
takes nothing from the GPU: the index is defined by the seeded generator).

The buckets are the rows' mixture components (256 of them, uneven sizes)
and the centroids the components' means, passed to the build; any centroid
set makes a valid IVF index, and the search's answer is defined over it.

* 1,000,000 x 1536 unit-norm rows, a random rotation (the oracle's QR of a
  seeded Gaussian), 10,000 queries, nprobe 8, eps0 = inf (exact within the
  probed buckets): for sampled queries the oracle's probe order and top-10
  over the probed rows, in the original space (a rotation keeps every
  distance), under the tie rule; queries tied at the probe boundary
  skipped.
* 5,000,000 x 768, bfloat16 and e4m3 copies (no rotation, so the oracle's
  e4m3 scales come from the rows themselves), 1,000 queries, nprobe 2,
  eps0 = inf: the scanned (decoded) distances with no rerank, and the f32
  rerank of the 40 best, against oracle.lowp on the sampled queries.
"""
import numpy as np
import pytest

import synth
from oracle import exact, lowp, rotation
from tests.parity import check_knn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pdx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_04422_amd as pdx
    return pdx


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _lists(lab, nlist):
    order = np.argsort(lab, kind="stable")
    bounds = np.searchsorted(lab[order], np.arange(nlist + 1))
    return [order[bounds[i]:bounds[i + 1]] for i in range(nlist)]


def _probe(c64, qv, nprobe):
    dist = exact.sqdist(c64, qv.astype(np.float64))
    order = np.lexsort((np.arange(dist.size), dist))
    tied = nprobe < dist.size and abs(dist[order[nprobe]] - dist[order[nprobe - 1]]) <= 1e-5 * dist[order[nprobe]]
    return order[:nprobe], tied


def test_ivf_1m_d1536_sampled_against_the_oracle(pdx):
    import torch
    x, q, mix = synth.workload("ivf_1m_d1536")
    n, d = x.shape
    lab = mix.labels(n)
    nlist, nprobe, k = mix.means.shape[0], 8, 10
    print(f"full-size IVF parity {n} x {d}, {q.shape[0]} queries, nlist {nlist}", flush=True)
    r64 = rotation.orthogonal_from_gaussian(np.random.default_rng(1536).standard_normal((d, d)))
    r32 = r64.astype(np.float32)
    c = mix.means.astype(np.float32)
    c_rot = rotation.rotate_rows(c, r32.astype(np.float64)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    ix = pdx.pdx_ivf_build(xd, nlist, None, None, rotation=torch.from_numpy(r32).cuda(),
                           centroids=torch.from_numpy(c_rot).cuda(), assign=torch.from_numpy(lab).cuda())
    gi, gd = pdx.pdx_search_ivf(ix, torch.from_numpy(q).cuda(), k, nprobe, eps0=float("inf"))
    gi, gd = _np(gi), _np(gd)
    del xd
    lists = _lists(lab, nlist)
    c64 = c.astype(np.float64)  # ||R q - R c|| = ||q - c||: the probe order in the original space
    checked = 0
    for i in np.random.default_rng(8).choice(q.shape[0], 12, replace=False):
        probe, tied = _probe(c64, q[i], nprobe)
        if tied:
            continue
        rows = np.concatenate([lists[p] for p in probe])
        wi, wd = exact.topk_by_dist_then_id(exact.sqdist(x[rows], q[i]), rows, k)
        check_knn(x, q[i:i + 1], gi[i:i + 1], gd[i:i + 1], wi[None], wd[None])
        checked += 1
    print(f"checked {checked} sampled queries", flush=True)
    assert checked >= 8


def test_lowp_5m_d768_sampled_against_the_oracle(pdx):
    import torch
    x, q, mix = synth.workload("lowp_5m_d768")
    q = q[:1000]
    n, d = x.shape
    lab = mix.labels(n)
    nlist, nprobe, k, r = mix.means.shape[0], 2, 10, 40
    print(f"full-size low-precision parity {n} x {d}, nlist {nlist}", flush=True)
    xd = torch.from_numpy(x).cuda()
    ix = pdx.pdx_ivf_build(xd, nlist, None, None, centroids=torch.from_numpy(mix.means.astype(np.float32)).cuda(),
                           assign=torch.from_numpy(lab).cuda(), lowp=("bf16", "fp8"))
    qd = torch.from_numpy(q).cuda()
    res = {}
    for dtype in ("bf16", "fp8"):
        res[dtype] = [_np(t) for t in pdx.pdx_search_ivf(ix, qd, k, nprobe, eps0=float("inf"), dtype=dtype,
                                                        rerank=-1)]
        res[dtype] += [_np(t) for t in pdx.pdx_search_ivf(ix, qd, k, nprobe, eps0=float("inf"), dtype=dtype,
                                                         rerank=r)]
    del xd, ix
    lists = _lists(lab, nlist)
    c64 = mix.means.astype(np.float64)
    scales = lowp.fp8_scales(x)  # over all 5M rows, as the build
    sample = [int(i) for i in np.random.default_rng(9).choice(q.shape[0], 6, replace=False)]
    probes = {}
    for i in sample:
        probe, tied = _probe(c64, q[i], nprobe)
        if not tied:
            probes[i] = probe
    need = np.unique(np.concatenate([lists[p] for pr in probes.values() for p in pr]))
    print(f"decoding {need.size} rows", flush=True)
    at = {int(v): j for j, v in enumerate(need)}
    dec = {"bf16": lowp.bf16_decode(lowp.bf16_encode(x[need])),
           "fp8": lowp.fp8_decode(lowp.fp8_encode_array(x[need], scales), scales)}
    checked = 0
    for i, probe in probes.items():
        rows = np.concatenate([lists[p] for p in probe])
        local = np.array([at[int(v)] for v in rows])
        for dtype in ("bf16", "fp8"):
            xdec = dec[dtype][local]
            si, sd, ri, rd = res[dtype]
            # scanned distances: the exact top-k over the decoded rows
            ad = exact.sqdist(xdec, q[i])
            wi, wd = exact.topk_by_dist_then_id(ad, rows, k)
            got = si[i]
            assert set(got.tolist()) <= set(rows.tolist())
            gam = np.array([ad[np.nonzero(rows == g)[0][0]] for g in got])
            assert np.all(np.abs(np.sort(gam) - wd) <= 1e-5 * wd[-1]), (dtype, i)
            assert np.all(np.abs(sd[i] - gam) <= 1e-5 * gam + 1e-30), (dtype, i)
            # rerank of the R best by the decoded distance, where the R-th is not tied
            srt = np.sort(ad)
            if srt.size > r and abs(srt[r] - srt[r - 1]) <= 1e-5 * srt[r]:
                continue
            order = np.lexsort((rows, ad))[:r]
            ex = exact.sqdist(x[rows[order]], q[i])
            wi, wd = exact.topk_by_dist_then_id(ex, rows[order], k)
            check_knn(x, q[i:i + 1], ri[i:i + 1], rd[i:i + 1], wi[None], wd[None])
            checked += 1
    print(f"checked {checked} (query, storage) pairs", flush=True)
    assert checked >= 6
