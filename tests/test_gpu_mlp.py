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

Prune bound:
* the pinball gradient and loss equal the oracle's;
* the multipliers the search computes after START equal the oracle's
  network evaluated on the oracle's inputs (START threshold, centroid
  distances), at every test point;
* traces of an exact search: targets and inputs equal the oracle's for
  every returned neighbour (NaN for the START bucket's);
* a huge bound gives the exact-within-buckets search bit for bit and a
  very negative one the START bucket's result, on every scan engine;
* constant bounds: the oracle's recall within 0.03; eps = 2 agrees with
  ADSampling's eps0 = 2;
* pinball training on the device, with its final bias calibration, covers
  its level of the training targets.
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
    return dict(x=x, q=q, c32=c32, lists=kmeans.lists_from_labels(lab, nlist), ix=ix, mix=mix, labels=lab)


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


# ---------------------------------------------------------------------------
# learned prune multiplier
# ---------------------------------------------------------------------------

def _net(entries, b3):
    parts = {"W1": np.zeros((64, 72)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
             "w3": np.zeros(64), "b3": np.array([b3])}
    for (name, idx), v in entries.items():
        parts[name][idx] = v
    return omlp.pack(parts).astype(np.float32)


def test_pinball_gradient_and_loss_match_oracle(pdx):
    th = _theta(11)
    st = pdx.MlpState(_dev(th))
    rng = np.random.default_rng(12)
    x = rng.standard_normal((300, omlp.F_IN)).astype(np.float32)
    th16 = omlp.fp16_round(th)
    z, _ = omlp.forward(th16, x)
    y = (z + rng.uniform(0.05, 1.0, 300) * rng.choice([-1.0, 1.0], 300)).astype(np.float32)  # no kinks
    g, loss = st.grad(_dev(x), _dev(y), 0.9, kind="pinball")
    g, loss = _np(g), float(_np(loss)[0])
    gw = omlp.grad(th16, x, y.astype(np.float64), 0.9, "pinball")
    np.testing.assert_allclose(g[:omlp.P_USED], gw[:omlp.P_USED], rtol=1e-3, atol=1e-3 * np.abs(gw).max())
    assert abs(loss - omlp.loss(th16, x, y.astype(np.float64), 0.9, "pinball")) <= 1e-4 * abs(loss)


def _probe_context(ivf, i, k, nprobe):
    """Oracle probe order, sorted probed centroid distances, START threshold,
    or None when a rounding-level tie decides the probe order."""
    x, q, c32, lists = ivf["x"], ivf["q"], ivf["c32"], ivf["lists"]
    q64 = q[i].astype(np.float64)
    cd = np.sort(exact.sqdist(c32, q64))
    if np.any(np.diff(cd[: nprobe + 1]) <= 1e-6 * cd[nprobe]):
        return None
    order = px.ivf_probe_order(c32, q64, nprobe)
    start = px.ivf_flat(x, lists, c32, q64, k, 1)[1]
    tau = start[-1] if np.isfinite(start[-1]) else np.inf
    return order, cd[:nprobe], tau


def test_prune_table_matches_oracle(pdx, ivf):
    import torch
    q = ivf["q"]
    nq, k, nprobe, dd = q.shape[0], 10, 12, 24  # D = 96: tests after 24, 48, 72 dimensions
    npt = pdx.ivf_test_points(96)
    assert npt == 3
    th = _theta(13, 0.05)
    th[omlp.P_USED - 1] = 1.0  # output bias: bounds around 1
    st = pdx.MlpState(_dev(th))
    th16 = omlp.fp16_round(th)
    for engine in (1, 2):
        table = torch.empty((nq, nprobe - 1, npt), dtype=torch.float32, device="cuda")
        pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, nprobe, prune_mlp=st, prune_scale=1.5, prune_table=table,
                           engine=engine)
        table = _np(table)
        checked = 0
        for i in range(nq):
            ctx = _probe_context(ivf, i, k, nprobe)
            if ctx is None:
                continue
            _, cd, tau = ctx
            want = omlp.prune_multipliers(th16, q[i].astype(np.float64), tau, cd, nprobe, dd, 1.5)
            np.testing.assert_allclose(table[i], want, rtol=2e-3)
            checked += 1
        assert checked >= nq - 3


def test_prune_traces_match_oracle(pdx, ivf):
    import torch
    x, q, c32, lists, labels = ivf["x"], ivf["q"], ivf["c32"], ivf["lists"], ivf["labels"]
    nq, k, nprobe, dd = q.shape[0], 10, 12, 24
    pf = torch.empty((nq, k, 72), dtype=torch.float32, device="cuda")
    pt = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    gi, gd = pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, nprobe, eps0=float("inf"), prune_trace=(pf, pt))
    pf, pt, gi, gd = _np(pf), _np(pt), _np(gi), _np(gd)
    want = [px.ivf_flat(x, lists, c32, q[i].astype(np.float64), k, nprobe) for i in range(nq)]
    check_knn(x, q, gi, gd, np.stack([w[0] for w in want]), np.stack([w[1] for w in want]))
    checked = samples = 0
    for i in range(nq):
        ctx = _probe_context(ivf, i, k, nprobe)
        if ctx is None or gi[i].tolist() != want[i][0].tolist():
            continue  # probe order or neighbour order decided by a rounding-level tie
        order, cd, tau = ctx
        rank = {int(b): r for r, b in enumerate(order)}
        q64 = q[i].astype(np.float64)
        targets = omlp.prune_targets(x, q64, want[i][0], want[i][1][-1], dd)
        for a, v in enumerate(want[i][0]):
            r = rank[int(labels[v])]
            if r == 0:  # START bucket: scanned whole, no sample
                assert np.isnan(pt[i, a]) and np.all(pf[i, a] == 0)
                continue
            np.testing.assert_allclose(pt[i, a], targets[a], rtol=1e-4, atol=1e-4)
            ref = omlp.prune_inputs(q64, tau, cd, r, nprobe)
            assert np.array_equal(pf[i, a, :64], q[i, :64])
            np.testing.assert_allclose(pf[i, a, 64:68], ref[64:68], rtol=1e-4)
            assert np.all(pf[i, a, 68:] == 0)
            samples += 1
        checked += 1
    assert checked >= nq - 5 and samples >= 100


def test_prune_extremes_on_every_engine(pdx, ivf):
    q, k = ivf["q"], 10
    keep_all = pdx.MlpState(_dev(_net({}, 60000.0)))   # eps = 6e4: nothing is dropped before D
    drop_all = pdx.MlpState(_dev(_net({}, -60000.0)))  # eps below -sqrt(c1): multiplier 0
    for engine, qpw in ((1, 1), (1, 4), (2, 0)):
        sched = dict(engine=engine, queries_per_wave=qpw)
        print(f"prune extremes engine {engine} qpw {qpw}", flush=True)
        base_i, base_d = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 24, eps0=float("inf"), **sched))
        gi, gd = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 24, prune_mlp=keep_all, **sched))
        assert np.array_equal(gi, base_i) and np.array_equal(gd, base_d)
        one_i, one_d = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 1, eps0=float("inf"), **sched))
        gi, gd = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 24, prune_mlp=drop_all, **sched))
        assert np.array_equal(gi, one_i) and np.array_equal(gd, one_d)


@pytest.mark.parametrize("eps", [0.5, 0.0])
def test_constant_bound_recall_band(pdx, ivf, eps):
    """A network whose output is the constant eps: the multiplier is
    ADSampling's shape (1 + eps/sqrt(c1))^2.  eps 0.5 keeps about 94% of
    IVF-flat's neighbours in the oracle's sequential search, eps 0 about
    85%.  The device tightens the threshold inside a bucket while the
    sequential search holds it per bucket, hence a band of 0.03."""
    x, q, c32, lists = ivf["x"], ivf["q"], ivf["c32"], ivf["lists"]
    nq, k, nprobe, dd = q.shape[0], 10, 12, 24
    th = _net({}, eps)
    st = pdx.MlpState(_dev(th))
    th16 = omlp.fp16_round(th)
    flat, seq = [], []
    for i in range(nq):
        q64 = q[i].astype(np.float64)
        order = px.ivf_probe_order(c32, q64, nprobe)
        cd = exact.sqdist(c32, q64)[order]
        start = px.ivf_flat(x, lists, c32, q64, k, 1)[1]
        tau = start[-1] if np.isfinite(start[-1]) else np.inf
        mult = omlp.prune_multipliers(th16, q64, tau, cd, nprobe, dd)
        seq.append(px.learned_ivf_search(x, lists, c32, q64, k, nprobe, mult, dd)[0])
        flat.append(px.ivf_flat(x, lists, c32, q64, k, nprobe)[0])
    flat, seq = np.stack(flat), np.stack(seq)
    r_seq = exact.recall_at_k(flat, seq)
    assert r_seq < 0.99  # the bound does prune neighbours: the band is a real check
    for engine in (1, 2):
        gi, gd = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, nprobe, prune_mlp=st, engine=engine))
        r_dev = exact.recall_at_k(flat, gi)
        print(f"eps {eps} engine {engine}: recall {r_dev:.4f}, oracle sequential {r_seq:.4f}", flush=True)
        assert abs(r_dev - r_seq) <= 0.03
        ok = gi >= 0
        true = ((x[gi[ok]].astype(np.float64) - q.astype(np.float64)[np.nonzero(ok)[0]]) ** 2).sum(1)
        np.testing.assert_allclose(gd[ok], true, rtol=1e-5)


def test_constant_bound_two_matches_adsampling(pdx, ivf):
    """eps = 2 from the network and ADSampling's eps0 = 2 use the same
    multipliers up to rounding: the results agree."""
    q, k = ivf["q"], 10
    st = pdx.MlpState(_dev(_net({}, 2.0)))
    for engine in (1, 2):
        ai, _ = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 12, eps0=2.0, engine=engine))
        gi, _ = (_np(t) for t in pdx.pdx_search_ivf(ivf["ix"], _dev(q), k, 12, prune_mlp=st, engine=engine))
        assert exact.recall_at_k(ai, gi) >= 0.99


def test_pinball_training_calibrates_the_bound(pdx, ivf):
    qt = ivf["mix"].queries(1500, 99)
    feats, targets, stats = pdx.learn.prune_traces(ivf["ix"], _dev(qt), 10, 12)
    assert stats["samples"] >= 2000 and stats["test_points"] == 3
    st, info = pdx.learn.train_prune_network(feats, targets, steps=1500, batch=2048, lr=3e-3, level=0.9)
    z = _np(st.forward(feats))
    t = _np(targets)
    frac = float(np.mean(t <= z))
    print(f"samples {t.size}, loss {info['loss_first']:.4f} -> {info['loss_last']:.4f}, covered {frac:.3f}",
          flush=True)
    assert info["loss_last"] < info["loss_first"]
    assert abs(frac - 0.9) <= 0.01  # the bias calibration (rounded to float16 in the deployed copy)
