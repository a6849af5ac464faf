"""What the trained prune network gains over the method without it.

On a small skewed-mixture IVF workload (D = 256, 7 ADSampling test
points), the prune network is trained on the device from the search's own
traces (training queries); its scale is picked on validation queries as the
cheapest that reaches the recall of plain ADSampling at the paper's
eps0 = 2.1 (Section 6.1) less 0.005; both are then run on fresh test
queries at the same nprobe, recall judged by the FP64 oracle's exact k-NN.
Asserted: the learned bound evaluates fewer (query, vector, dimension)
values than ADSampling as the paper configures it (the library's counters),
at a recall no more than 0.01 below.  This is all it gains: a single eps0
retuned to the same recall evaluates as few values or fewer on this
workload, so the per-(query, bucket) inputs add nothing beyond lowering the
bound.
"""
import numpy as np
import pytest

import synth
from oracle import exact

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


def test_trained_prune_bound_evaluates_fewer_values(pdx, oracle_c):
    import torch
    k, nlist, nprobe = 10, 256, 16
    mix = synth.skewed_mixture(256, 32, 32.0, 4.0, 42)
    x = mix.data(100_000)
    qt = mix.queries(4000, 43)
    qv, qs = mix.queries(500, 45), mix.queries(1000, 44)
    rng = np.random.default_rng(42)
    g = rng.standard_normal((x.shape[1], x.shape[1]))
    init = rng.choice(x.shape[0], nlist, replace=False).astype(np.int64)
    print("learned gain: building the index", flush=True)
    ix = pdx.pdx_ivf_build(_dev(x), nlist, _dev(g), _dev(init), kmeans_iters=10)
    tv = oracle_c.knn_exact_c(x, qv, k)[0]
    ts = oracle_c.knn_exact_c(x, qs, k)[0]
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")

    def run(q, **kw):
        cnt.zero_()
        ids, _ = pdx.pdx_search_ivf(ix, _dev(q), k, nprobe, counters=cnt, **kw)
        c = cnt.cpu().numpy()
        return ids.cpu().numpy(), float(c[0] + c[2]) / q.shape[0]

    print("learned gain: traces and training", flush=True)
    feats, targets, stats = pdx.learn.prune_traces(ix, _dev(qt), k, nprobe)
    assert stats["samples"] > 1000
    net, info = pdx.learn.train_prune_network(feats, targets, level=0.95, steps=1500)
    assert info["loss_last"] < info["loss_first"]

    plain_v = exact.recall_at_k(tv, run(qv, eps0=2.1)[0])
    target = plain_v - 0.005
    pick = None
    for sc in [round(0.2 + 0.1 * i, 2) for i in range(30)]:  # increasing recall
        ids, _ = run(qv, prune_mlp=net, prune_scale=sc)
        if exact.recall_at_k(tv, ids) >= target:
            pick = sc
            break
    assert pick is not None, "no scale reaches plain ADSampling's validation recall"
    p_ids, p_work = run(qs, eps0=2.1)
    l_ids, l_work = run(qs, prune_mlp=net, prune_scale=pick)
    p_rec, l_rec = exact.recall_at_k(ts, p_ids), exact.recall_at_k(ts, l_ids)
    print(f"plain eps0=2.1: recall {p_rec:.4f}, {p_work:.0f} values/query; "
          f"learned scale {pick}: recall {l_rec:.4f}, {l_work:.0f} values/query", flush=True)
    assert l_rec >= p_rec - 0.01
    assert l_work < p_work
