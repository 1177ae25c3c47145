"""Pins of the FP64 predictor reference (forward, backward, Adam) by routes
independent of its own code: central finite differences, closed forms for
zero weights and single samples, and the defining property of Adam's first step."""
import numpy as np
import pytest

from oracle import mlp


def rand_w(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, mlp.NW)


def rand_x(seed, n):
    rng = np.random.default_rng(seed + 1000)
    return rng.uniform(0, 12, size=(n, 3))


def test_parameter_count():
    assert mlp.NW == 1217


@pytest.mark.parametrize("seed", range(3))
def test_backward_matches_central_differences(seed):
    w = rand_w(seed)
    X = rand_x(seed, 9)
    T = np.random.default_rng(seed + 7).uniform(0, 10, 9)
    y, cache = mlp.forward(w, X)
    # keep away from ReLU kinks, where the derivative is one-sided
    _, z1, _, z2, _ = cache
    assert np.abs(z1).min() > 1e-4 and np.abs(z2).min() > 1e-4
    L, dy = mlp.mse(y, T)
    g = mlp.backward(w, cache, dy)
    h = 1e-6
    num = np.empty_like(w)
    for p in range(w.size):
        wp = w.copy(); wp[p] += h
        wm = w.copy(); wm[p] -= h
        num[p] = (mlp.mse(mlp.forward(wp, X)[0], T)[0] - mlp.mse(mlp.forward(wm, X)[0], T)[0]) / (2 * h)
    scale = np.abs(g).max()
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-6 * scale)


def test_zero_weights_give_last_bias_and_no_first_layer_gradient():
    w = np.zeros(mlp.NW)
    w[-1] = 3.25
    X = rand_x(0, 5)
    y, cache = mlp.forward(w, X)
    np.testing.assert_array_equal(y, np.full(5, 3.25))
    g = mlp.backward(w, cache, np.ones(5))
    W1, b1, W2, b2, w3, b3 = mlp.unpack(g)
    assert not W1.any() and not b1.any() and not W2.any() and not b2.any()
    assert b3 == 5.0


def test_single_sample_layer_gradients_are_outer_products():
    w = rand_w(4)
    x = rand_x(4, 1)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(w)
    # forward by hand, one sample
    z1 = np.array([sum(W1[o, i] * x[0, i] for i in range(3)) + b1[o] for o in range(32)])
    h1 = np.where(z1 > 0, z1, 0.0)
    z2 = np.array([sum(W2[o, i] * h1[i] for i in range(32)) + b2[o] for o in range(32)])
    h2 = np.where(z2 > 0, z2, 0.0)
    y = sum(w3[i] * h2[i] for i in range(32)) + b3
    yy, cache = mlp.forward(w, x)
    assert abs(yy[0] - y) <= 1e-12 * (1 + abs(y))
    g = mlp.unpack(mlp.backward(w, cache, np.array([1.0])))
    dz2 = w3 * (z2 > 0)
    np.testing.assert_allclose(g[4], h2, rtol=1e-14)
    np.testing.assert_allclose(g[2], np.outer(dz2, h1), rtol=1e-13, atol=1e-15)
    dz1 = np.array([sum(W2[o, i] * dz2[o] for o in range(32)) for i in range(32)]) * (z1 > 0)
    np.testing.assert_allclose(g[0], np.outer(dz1, x[0]), rtol=1e-12, atol=1e-15)


def test_first_adam_step_moves_each_weight_by_lr_against_gradient_sign():
    w = rand_w(1)
    g = np.random.default_rng(2).normal(size=w.size)
    w1, m, v = mlp.adam_step(w, g, np.zeros_like(w), np.zeros_like(w), 1, 1e-3)
    # with bias correction, m_hat = g and v_hat = g^2, so the step is lr*g/(|g|+eps)
    np.testing.assert_allclose(w - w1, 1e-3 * g / (np.abs(g) + mlp.EPS), rtol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 10, size=(2048, 3))
    T = 0.3 * X[:, 0] + 0.9 * X[:, 1] - 0.2 * np.maximum(X[:, 2] - 3, 0)
    w0 = rand_w(6, scale=0.2)
    w0[-1] = T.mean()
    _, losses = mlp.train(X, T, w0, epochs=8, lr=3e-3, batch=256)
    assert losses[-1] < 0.2 * losses[0]
    assert np.mean(np.diff(losses)) < 0


def test_pinball_gradient_and_minimiser():
    """Pinball loss: gradient by central differences away from kinks, and a
    constant predictor trained on it settles at the q-quantile of the targets."""
    rng = np.random.default_rng(8)
    y = rng.normal(size=50)
    t = rng.normal(size=50)
    q = 0.8
    L, g = mlp.pinball(y, t, q)
    h = 1e-7
    for i in range(0, 50, 7):
        yp = y.copy(); yp[i] += h
        ym = y.copy(); ym[i] -= h
        num = (mlp.pinball(yp, t, q)[0] - mlp.pinball(ym, t, q)[0]) / (2 * h)
        assert abs(num - g[i]) < 1e-6
    T = rng.exponential(2.0, 3000)
    X = rng.uniform(0, 5, size=(3000, 3))
    w0 = np.zeros(mlp.NW)
    w, _ = mlp.train(X, T, w0, epochs=600, lr=0.1, batch=3000, quantile=0.9)
    assert not w[:-1].any()
    assert abs(w[-1] - np.quantile(T, 0.9)) < 0.05


def test_features_are_log2_of_one_plus_each_count_in_order():
    """features(len, ub, mx) per row is (log2(1+len), log2(1+ub), log2(1+mx)):
    counts one below a power of two give exact integers, so a wrong base, a
    missing +1 or swapped columns all change these values."""
    got = mlp.features([0, 1, 3, 1023], [7, 15, 0, 1], [1, 0, 255, 3])
    want = np.array([[0.0, 3.0, 1.0],
                     [1.0, 4.0, 0.0],
                     [2.0, 0.0, 8.0],
                     [10.0, 1.0, 2.0]])
    assert got.shape == (4, 3) and got.dtype == np.float64
    np.testing.assert_array_equal(got, want)
    # between powers of two the feature is strictly between the neighbours' integers
    f = mlp.features([2, 4, 5], [2, 4, 5], [2, 4, 5])
    assert (f[:, 0] == f[:, 1]).all() and (f[:, 1] == f[:, 2]).all()
    assert 1.0 < f[0, 0] < 2.0 and 2.0 < f[1, 0] < f[2, 0] < 3.0
    np.testing.assert_allclose(2.0 ** f[:, 0], [3.0, 5.0, 6.0], rtol=1e-15)
