"""Pins of the FP64 reference of the learned bracket predictor (oracle/mlp_ref.py)."""

import numpy as np

from oracle import mlp_ref as M


def rand_params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0.0, scale, M.NPARAMS)


def test_parameter_count():
    assert M.NPARAMS == 4482
    p = rand_params(1)
    assert np.array_equal(M.pack(*M.unpack(p)), p)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    p = rand_params(3)
    z = rng.normal(size=(17, 2))
    ystar = rng.normal(size=(17, 2))
    L, g = M.loss_and_grad(p, z, ystar, alpha=4.0)
    idx = rng.choice(M.NPARAMS, 300, replace=False)
    idx = np.concatenate([idx, [0, 1, 127, 128, 191, 192, 4287, 4288, 4351, 4352, 4479, 4480, 4481]])
    h = 1e-6
    for i in idx:
        dp = np.zeros_like(p)
        dp[i] = h
        fd = (M.loss_and_grad(p + dp, z, ystar, 4.0)[0] - M.loss_and_grad(p - dp, z, ystar, 4.0)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), i


def test_zero_weights_give_bias_and_zero_hidden_gradients():
    p = np.zeros(M.NPARAMS)
    W1, b1, W2, b2, W3, b3 = M.unpack(p)
    b3 = np.array([0.25, -1.5])
    p = M.pack(W1, b1, W2, b2, W3, b3)
    z = np.random.default_rng(4).normal(size=(9, 2))
    y, _ = M.forward(p, z)
    assert np.array_equal(y, np.tile(b3, (9, 1)))
    _, g = M.loss_and_grad(p, z, np.zeros((9, 2)), 3.0)
    gW1, gb1, gW2, gb2, gW3, gb3 = M.unpack(g)
    # with W3 = 0 no gradient reaches the hidden layers; with h2 = 0, gW3 = 0
    assert not gW1.any() and not gb1.any() and not gW2.any() and not gb2.any() and not gW3.any()
    # e0 = 0.25 > 0 (weight 3), e1 = -1.5 < 0 (weight 3): gb3 = w e (mean over the batch)
    assert np.allclose(gb3, [3 * 0.25, 3 * -1.5])


def test_network_is_odd_without_biases():
    W1, b1, W2, b2, W3, b3 = M.unpack(rand_params(5))
    p = M.pack(W1, 0 * b1, W2, 0 * b2, W3, 0 * b3)
    z = np.random.default_rng(6).normal(size=(11, 2))
    assert np.allclose(M.forward(p, -z)[0], -M.forward(p, z)[0], rtol=0, atol=1e-15)


def test_asymmetric_weights_select_unsafe_side():
    p = np.zeros(M.NPARAMS)
    W1, b1, W2, b2, W3, b3 = M.unpack(p)
    z = np.zeros((1, 2))
    # prediction y = b3; targets chosen so e0 > 0 and e1 > 0: only e0 is unsafe
    L, _ = M.loss_and_grad(M.pack(W1, b1, W2, b2, W3, np.array([1.0, 1.0])), z, np.zeros((1, 2)), 5.0)
    assert np.isclose(L, 0.5 * (5.0 + 1.0))
    L, _ = M.loss_and_grad(M.pack(W1, b1, W2, b2, W3, np.array([-1.0, -1.0])), z, np.zeros((1, 2)), 5.0)
    assert np.isclose(L, 0.5 * (1.0 + 5.0))


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3])
    p, m, s = M.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g))


def test_targets_and_bracket_roundtrip():
    t0 = np.array([0.0, 0.5, 2.0])
    t1 = np.array([1.0, 2.0, 7.0])
    y = M.targets(t0, t1)
    b0, b1 = M.bracket_from_outputs(y, 0.0, 0.0)
    assert np.allclose(b0, t0) and np.allclose(b1, t1)
    b0, b1 = M.bracket_from_outputs(y, 0.1, 0.05)
    assert np.all(b1 > t1) and np.all(b0 <= t0)


def test_activation_shape():
    # phi(a) = u (3 - u^2) / 2, u = clamp(a / 1.5, -1, 1): odd, slope 1 at 0,
    # +-1 from |a| = 1.5 on with a vanishing slope there, increasing, and its
    # derivative (returned beside it) is the slope of its values
    a = np.linspace(-4.0, 4.0, 8001)
    h, d = M.phi(a)
    assert np.array_equal(M.phi(-a)[0], -h)
    assert M.phi(0.0)[0] == 0.0 and M.phi(0.0)[1] == 1.0
    assert np.all(h[a >= 1.5] == 1.0) and np.all(h[a <= -1.5] == -1.0)
    assert np.all(d[np.abs(a) >= 1.5] == 0.0)
    assert np.all(np.diff(h) >= 0.0) and np.all(np.abs(h) <= 1.0)
    eps = 1e-6
    fd = (M.phi(a + eps)[0] - M.phi(a - eps)[0]) / (2 * eps)
    assert np.max(np.abs(fd - d)) <= 1e-6
    # the cubic through (0, 0) and (1.5, 1) with slopes 1 and 0 there
    assert np.isclose(M.phi(0.75)[0], 0.6875) and np.isclose(M.phi(0.75)[1], 0.75)


def test_first_layer_clamp():
    a = np.array([-3.0, -1.0, -0.999, -0.25, 0.0, 0.5, 0.999, 1.0, 2.0])
    h, d = M.hard_clamp(a)
    assert np.array_equal(h, [-1.0, -1.0, -0.999, -0.25, 0.0, 0.5, 0.999, 1.0, 1.0])
    assert np.array_equal(d, [0, 0, 1, 1, 1, 1, 1, 0, 0])
    # the network's first layer is the clamp: with W2 = I-like weights read out
    # through W3, y follows phi(clamp(W1 z + b1)) by hand on one unit
    p = np.zeros(M.NPARAMS)
    W1, b1, W2, b2, W3, b3 = M.unpack(p)
    W1[0] = [2.0, 0.0]
    W2[0, 0] = 1.0
    W3[0, 0] = 1.0
    p = M.pack(W1, b1, W2, b2, W3, b3)
    z = np.array([[0.3, 5.0], [0.9, -1.0], [-4.0, 0.0]])
    y, _ = M.forward(p, z)
    expect = M.phi(np.clip(2.0 * z[:, 0], -1, 1))[0]
    assert np.allclose(y[:, 0], expect) and np.all(y[:, 1] == 0.0)
