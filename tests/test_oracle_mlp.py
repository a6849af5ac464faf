"""Pins for the network oracle.  CPU only.

* a hand-worked network (weights chosen so every unit is computed by hand);
* analytic gradient vs central finite differences (1e-6);
* the loss is the weighted binary cross-entropy: a planted sign error in
  dL/dz fails the finite-difference check.
"""
import numpy as np

from oracle import mlp


def test_hand_worked_forward():
    parts = {"W1": np.zeros((64, 72)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
             "w3": np.zeros(64), "b3": np.array([0.5])}
    parts["W1"][0, 0] = 2.0      # a1[0] = 2 x0
    parts["W1"][1, 1] = -1.0     # a1[1] = -x1 (relu kills it for x1 > 0)
    parts["W2"][0, 0] = 3.0      # a2[0] = 3 h1[0] + 1
    parts["b2"][0] = 1.0
    parts["W2"][1, 1] = 5.0      # a2[1] = 5 h1[1]
    parts["w3"][0] = 0.25
    parts["w3"][1] = 7.0
    th = mlp.pack(parts)
    x = np.zeros((2, 72))
    x[0, 0], x[0, 1] = 1.5, 2.0   # h1 = (3, 0) -> h2 = (10, 0) -> z = 2.5 + 0.5 = 3
    x[1, 0], x[1, 1] = -1.0, -0.4  # h1 = (0, 0.4) -> h2 = (1, 2) -> z = 0.25 + 14 + 0.5 = 14.75
    z, _ = mlp.forward(th, x)
    np.testing.assert_allclose(z, [3.0, 14.75], rtol=0, atol=1e-12)


def _random_problem(seed=0, n=40):
    rng = np.random.default_rng(seed)
    th = rng.standard_normal(mlp.P_PAD) * 0.2
    th[mlp.P_USED:] = 0
    x = rng.standard_normal((n, mlp.F_IN))
    y = (rng.random(n) < 0.4).astype(np.float64)
    return th, x, y


def test_gradient_matches_finite_differences():
    th, x, y = _random_problem()
    g = mlp.grad(th, x, y, 3.0)
    idx = list(np.random.default_rng(1).choice(mlp.P_USED, 60, replace=False)) + [mlp.P_USED - 1, 0, 4608]
    num = mlp.numeric_grad(th, x, y, 3.0, idx)
    np.testing.assert_allclose(g[idx], num, rtol=1e-5, atol=1e-7)
    assert np.all(g[mlp.P_USED:] == 0)


def test_planted_sign_error_is_caught():
    th, x, y = _random_problem(2)
    good = mlp.grad(th, x, y, 2.0)
    bad = mlp.grad(th, x, 1.0 - y, 2.0)  # labels flipped = wrong sign on the data term
    idx = list(range(4608, 4608 + 16))
    num = mlp.numeric_grad(th, x, y, 2.0, idx)
    assert np.allclose(good[idx], num, rtol=1e-5, atol=1e-7)
    assert not np.allclose(bad[idx], num, rtol=1e-3, atol=1e-6)


def test_loss_decreases_along_negative_gradient():
    th, x, y = _random_problem(3)
    l0 = mlp.loss(th, x, y, 1.5)
    th2 = th - 0.05 * mlp.grad(th, x, y, 1.5)
    assert mlp.loss(th2, x, y, 1.5) < l0


# ---------------------------------------------------------------------------
# pinball (quantile) loss of the prune-multiplier network
# ---------------------------------------------------------------------------

def _constant_net(b3):
    parts = {"W1": np.zeros((64, 72)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
             "w3": np.zeros(64), "b3": np.array([b3])}
    return mlp.pack(parts)


def test_pinball_hand_worked():
    th = _constant_net(1.0)  # z = 1 for every sample
    x = np.zeros((3, 72))
    y = np.array([3.0, 0.0, 1.0])  # u = y - z = 2, -1, 0
    # level 0.9: 2 * 0.9 + (-1) * (0.9 - 1) + 0 = 1.9, mean 1.9 / 3
    assert abs(mlp.loss(th, x, y, 0.9, "pinball") - 1.9 / 3) < 1e-15
    # dL/db3 = mean([z > y] - 0.9) = (-0.9 + 0.1 - 0.9) / 3
    g = mlp.grad(th, x, y, 0.9, "pinball")
    assert abs(g[mlp.P_USED - 1] - (-1.7 / 3)) < 1e-15


def test_pinball_minimiser_is_the_quantile():
    y = np.random.default_rng(5).standard_normal(1001) * 2.0 + 0.3
    x = np.zeros((y.size, 72))
    for level in (0.5, 0.9, 0.98):
        q = np.quantile(y, level, method="inverted_cdf")
        lq = mlp.loss(_constant_net(q), x, y, level, "pinball")
        for dz in (-0.05, -0.01, 0.01, 0.05):
            assert mlp.loss(_constant_net(q + dz), x, y, level, "pinball") >= lq
        # the share of targets at or below the estimate is the level
        assert abs(np.mean(y <= q) - level) <= 1.0 / y.size


def _random_regression(seed=6, n=40):
    rng = np.random.default_rng(seed)
    th = rng.standard_normal(mlp.P_PAD) * 0.2
    th[mlp.P_USED:] = 0
    x = rng.standard_normal((n, mlp.F_IN))
    y = rng.standard_normal(n) * 2.0
    return th, x, y


def test_pinball_gradient_matches_finite_differences():
    th, x, y = _random_regression()
    z, _ = mlp.forward(th, x)
    assert np.min(np.abs(z - y)) > 1e-3  # no sample at a kink
    g = mlp.grad(th, x, y, 0.85, "pinball")
    idx = list(np.random.default_rng(7).choice(mlp.P_USED, 60, replace=False)) + [mlp.P_USED - 1, 0, 4608]
    num = mlp.numeric_grad(th, x, y, 0.85, idx, kind="pinball")
    np.testing.assert_allclose(g[idx], num, rtol=1e-5, atol=1e-7)


def test_pinball_planted_level_swap_is_caught():
    th, x, y = _random_regression(8)
    good = mlp.grad(th, x, y, 0.9, "pinball")
    bad = mlp.grad(th, x, y, 0.1, "pinball")  # under- and over-estimates weighted the wrong way round
    idx = list(range(4608, 4608 + 16)) + [mlp.P_USED - 1]
    num = mlp.numeric_grad(th, x, y, 0.9, idx, kind="pinball")
    assert np.allclose(good[idx], num, rtol=1e-5, atol=1e-7)
    assert not np.allclose(bad[idx], num, rtol=1e-3, atol=1e-6)


def test_prune_inputs_hand_worked():
    q = np.arange(1.0, 101.0)  # D = 100: the first 64 coordinates are 1 .. 64
    cd = np.array([2.0, 4.0, 8.0, 16.0])
    x = mlp.prune_inputs(q, 6.0, cd, 2, 4)
    np.testing.assert_array_equal(x[:64], np.arange(1.0, 65.0))
    # tau/d_2 = 0.75, d_2/d_0 = 4, tau/d_0 = 3, log2(2)/log2(4) = 0.5
    np.testing.assert_allclose(x[64:68], [0.75, 4.0, 3.0, 0.5], rtol=0, atol=1e-15)
    assert np.all(x[68:] == 0)
    # short queries are zero-padded; an infinite START threshold clamps to 1e4
    x = mlp.prune_inputs(np.ones(10), np.inf, cd, 1, 4)
    assert np.all(x[:10] == 1) and np.all(x[10:64] == 0)
    assert x[64] == 1e4 and x[66] == 1e4 and x[65] == 2.0


def test_prune_multipliers_follow_the_network():
    th = _constant_net(2.0)  # z = 2 for every rank
    m = mlp.prune_multipliers(th, np.ones(96), 5.0, np.array([1.0, 2.0, 3.0]), 3, 32, scale=1.5)
    assert m.shape == (2, 2)  # ranks 1, 2; test points after 32 and 64 of 96 dimensions
    # eps = 3: (1 + 3/sqrt(32))^2 and (1 + 3/sqrt(64))^2
    np.testing.assert_allclose(m[0], [(1 + 3 / np.sqrt(32)) ** 2, (1 + 3 / 8) ** 2], rtol=1e-15)
    np.testing.assert_array_equal(m[0], m[1])
    assert mlp.test_points(96, 32) == [32, 64] and mlp.test_points(97, 32) == [32, 64, 96]
    # a bound below -sqrt(c1) gives multiplier 0; a huge one is capped
    assert mlp.multiplier(-10.0, 64) == 0.0 and mlp.multiplier(1e20, 64) == 1e30
    # eps0 itself reproduces ADSampling's multiplier
    assert mlp.multiplier(2.1, 50) == (1.0 + 2.1 / np.sqrt(50)) ** 2


def test_prune_targets_brute_force():
    rng = np.random.default_rng(9)
    xr = rng.standard_normal((30, 70))
    q = rng.standard_normal(70)
    ids = np.array([3, 17, 29])
    t = mlp.prune_targets(xr, q, ids, 2.5, 16)
    assert t.shape == (3,)  # test points after 16, 32, 48, 64 of 70 dimensions
    for a, i in enumerate(ids):
        need = []
        for c1 in (16, 32, 48, 64):
            part = sum((xr[i, j] - q[j]) ** 2 for j in range(c1))
            need.append((np.sqrt(part * 70 / (c1 * 2.5)) - 1) * np.sqrt(c1))
        assert abs(t[a] - max(need)) < 1e-12
        # the target is the smallest bound that keeps the id at every test point
        for c1 in (16, 32, 48, 64):
            part = sum((xr[i, j] - q[j]) ** 2 for j in range(c1))
            assert part * 70 / c1 <= 2.5 * mlp.multiplier(t[a], c1) * (1 + 1e-12)
