"""GPU checks of the learned early-termination network and the checkpoint
traces it is trained on.

* forward logits, loss and gradient of the device kernels equal the FP64
  oracle evaluated on the same float16-rounded weights (1e-3);
* Adam training on the device lowers the loss and learns a separable rule;
* checkpoint traces of an exact (eps0 = inf) search: the k-best ids after
  2, 4, 8, 16, 32 probed buckets equal the oracle's IVF-flat with that
  nprobe, and the recorded inputs equal the oracle's (query coordinates,
  threshold and centroid-distance ratios);
* a network that never stops gives the plain search's result bit for bit;
  one that always stops gives the result of probing 2 buckets.
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


def test_checkpoint_traces_match_oracle(pdx, ivf):
    import torch
    x, q, c32, lists = ivf["x"], ivf["q"], ivf["c32"], ivf["lists"]
    nq, k, nprobe = q.shape[0], 10, 40
    tf = torch.empty((nq, 5, 72), dtype=torch.float32, device="cuda")
    ti = torch.empty((nq, 5, k), dtype=torch.int64, device="cuda")
    pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, nprobe, eps0=float("inf"), trace=(tf, ti))
    tf, ti = _np(tf), _np(ti)
    q64 = q.astype(np.float64)
    for c, cp in enumerate((2, 4, 8, 16, 32)):
        want = [px.ivf_flat(x, lists, c32, q64[i], k, cp) for i in range(nq)]
        check_knn(x, q, ti[:, c], np.stack([exact.sqdist(x[ti[i, c]], q[i]) for i in range(nq)]),
                  np.stack([w[0] for w in want]), np.stack([w[1] for w in want]))
        for i in range(nq):
            cd = np.sort(exact.sqdist(c32, q64[i]))
            tau = want[i][1][-1]
            ref = [tau / cd[cp], cd[cp] / cd[0], cd[nprobe - 1] / cd[0], tau / cd[0], np.log2(cp) / np.log2(nprobe)]
            np.testing.assert_allclose(tf[i, c, :64], q[i, :64], rtol=0, atol=0)
            np.testing.assert_allclose(tf[i, c, 64:69], np.minimum(ref, 1e4), rtol=1e-4)
            assert np.all(tf[i, c, 69:] == 0)


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
    two_i, two_d = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 2, eps0=float("inf")))
    ai, ad = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 24, eps0=float("inf"),
                                                  mlp=pdx.MlpState(_dev(always)), mlp_threshold=0.5))
    assert np.array_equal(ai, two_i) and np.array_equal(ad, two_d)
