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
