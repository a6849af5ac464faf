"""GPU checks of the learned early-termination network and the checkpoint
traces it is trained on.

* forward logits, loss and gradient of the device kernels equal the FP64
  oracle evaluated on the same float16-rounded weights (1e-3);
* Adam training on the device lowers the loss and learns a separable rule;
* budget traces of an exact (eps0 = inf) search: the result equals the
  oracle's IVF-flat, the recorded "buckets needed" is 1 + the largest
  probe rank (oracle order) holding a returned id, and the recorded inputs
  for every r equal the oracle's (query coordinates, START threshold and
  centroid-distance ratios);
* a network that never fires gives the plain search's result bit for bit;
  one that always fires gives the result of probing 1 bucket.
"""
import numpy as np
import pytest

import synth
from oracle import exact, kmeans, mlp as omlp, pdxearch as px
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


def _theta(seed, scale=0.15):
    th = (np.random.default_rng(seed).standard_normal(omlp.P_PAD) * scale).astype(np.float32)
    th[omlp.P_USED:] = 0
    return th


def test_forward_loss_and_gradient_match_oracle(pdx):
    th = _theta(1)
    st = pdx.MlpState(_dev(th))
    rng = np.random.default_rng(2)
    x = rng.standard_normal((300, omlp.F_IN)).astype(np.float32)
    y = (rng.random(300) < 0.35).astype(np.float32)
    z = _np(st.forward(_dev(x)))
    th16 = omlp.fp16_round(th)
    zw, _ = omlp.forward(th16, x)
    np.testing.assert_allclose(z, zw, rtol=1e-3, atol=1e-3)
    g, loss = st.grad(_dev(x), _dev(y), 2.5)
    g, loss = _np(g), float(_np(loss)[0])
    gw = omlp.grad(th16, x, y, 2.5)
    np.testing.assert_allclose(g[:omlp.P_USED], gw[:omlp.P_USED], rtol=1e-3, atol=1e-3 * np.abs(gw).max())
    assert np.all(g[omlp.P_USED:] == 0)
    assert abs(loss - omlp.loss(th16, x, y, 2.5)) <= 1e-4 * abs(loss)


def test_training_learns_a_separable_rule(pdx):
    import torch
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4000, omlp.F_IN)).astype(np.float32)
    y = ((x[:, 0] - 0.5 * x[:, 1] + 0.3 * x[:, 64]) > 0.2).astype(np.float32)
    st = pdx.MlpState(_dev(_theta(4, 0.1)))
    xd, yd = _dev(x), _dev(y)
    loss = torch.empty(1, device="cuda")
    losses = []
    for step in range(1, 301):
        st.train_step(xd, yd, 1.0, 3e-3, step, loss=loss)
        if step in (1, 300):
            losses.append(float(_np(loss)[0]))
    z = _np(st.forward(xd))
    acc = np.mean((z > 0) == (y > 0.5))
    print(f"loss {losses[0]:.4f} -> {losses[1]:.4f}, accuracy {acc:.4f}", flush=True)
    assert losses[1] < 0.5 * losses[0]
    assert acc >= 0.95


@pytest.fixture(scope="module")
def ivf(pdx):
    n, d, nlist = 30_000, 96, 60
    mix = synth.anisotropic_unit_mixture(d, 24, 13)
    x = mix.data(n)
    q = mix.queries(50)
    init = np.random.default_rng(5).choice(n, nlist, replace=False)
    c, lab, _ = kmeans.lloyd(x, init, 6)
    c32 = c.astype(np.float32)
    ix = pdx.pdx_ivf_build(_dev(x), nlist, None, None, centroids=_dev(c32), assign=_dev(lab.astype(np.int32)))
    return dict(x=x, q=q, c32=c32, lists=kmeans.lists_from_labels(lab, nlist), ix=ix)


def test_budget_traces_match_oracle(pdx, ivf):
    import torch
    x, q, c32, lists = ivf["x"], ivf["q"], ivf["c32"], ivf["lists"]
    nq, k, nprobe = q.shape[0], 10, 12
    tf = torch.empty((nq, nprobe, 72), dtype=torch.float32, device="cuda")
    need = torch.empty(nq, dtype=torch.int32, device="cuda")
    gi, gd = pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, nprobe, eps0=float("inf"), trace=(tf, need))
    tf, need, gi, gd = _np(tf), _np(need), _np(gi), _np(gd)
    q64 = q.astype(np.float64)
    labels = np.empty(x.shape[0], np.int64)
    for l, rows in enumerate(lists):
        labels[rows] = l
    want = [px.ivf_flat(x, lists, c32, q64[i], k, nprobe) for i in range(nq)]
    check_knn(x, q, gi, gd, np.stack([w[0] for w in want]), np.stack([w[1] for w in want]))
    checked = 0
    for i in range(nq):
        cd_all = exact.sqdist(c32, q64[i])
        cd = np.sort(cd_all)
        if np.any(np.diff(cd[: nprobe + 1]) <= 1e-6 * cd[nprobe]):
            continue  # probe order decided by a rounding-level tie
        order = px.ivf_probe_order(c32, q64[i], nprobe)
        rank = {int(b): r for r, b in enumerate(order)}
        assert need[i] == 1 + max(rank[int(labels[v])] for v in gi[i] if v >= 0)
        start = px.ivf_flat(x, lists, c32, q64[i], k, 1)[1]
        tau = start[-1] if np.isfinite(start[-1]) else np.inf
        for r in range(1, nprobe):
            ref = np.array([tau / cd[r], cd[r] / cd[0], cd[nprobe - 1] / cd[0], tau / cd[0],
                            np.log2(r) / np.log2(nprobe)])
            np.testing.assert_allclose(tf[i, r - 1, :64], q[i, :64], rtol=0, atol=0)
            np.testing.assert_allclose(tf[i, r - 1, 64:69], np.minimum(ref, 1e4), rtol=1e-4)
            assert np.all(tf[i, r - 1, 69:] == 0)
        assert np.all(tf[i, nprobe - 1] == 0)
        checked += 1
    assert checked >= nq - 3


def test_abstaining_and_always_stopping_networks(pdx, ivf):
    q, k = ivf["q"], 10
    never = np.zeros(omlp.P_PAD, np.float32)
    never[omlp.P_USED - 1] = -50.0  # b3: logit -50, never above the threshold
    always = never.copy()
    always[omlp.P_USED - 1] = 50.0
    for eps in (float("inf"), 2.1):
        base_i, base_d = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 24, eps0=eps))
        ni, nd = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 24, eps0=eps,
                                                      mlp=pdx.MlpState(_dev(never)), mlp_threshold=0.5))
        if eps == float("inf"):
            assert np.array_equal(ni, base_i) and np.array_equal(nd, base_d)
        else:
            assert exact.recall_at_k(base_i, ni) >= 0.99
    for engine in (1, 2):  # each scan engine: a budget of 1 bucket == probing 1
        one_i, one_d = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 1, eps0=float("inf"),
                                                            engine=engine))
        ai, ad = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 24, eps0=float("inf"), engine=engine,
                                                      mlp=pdx.MlpState(_dev(always)), mlp_threshold=0.5))
        assert np.array_equal(ai, one_i) and np.array_equal(ad, one_d)
