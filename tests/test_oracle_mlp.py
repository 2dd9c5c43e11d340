"""Pins of the learned-predictor oracle (CPU): each check is fixed by
mathematics independent of the oracle's own formulas (finite differences,
closed forms, identities, bit patterns)."""
import numpy as np
import pytest

from oracle import mlp


def _rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(mlp.N_PARAMS) * scale


def test_parameter_count_and_layout():
    assert mlp.N_PARAMS == 5379
    p = np.arange(mlp.N_PARAMS, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    assert W1.shape == (64, 15) and W1[1, 0] == 15 and b1[0] == 960
    assert W2[0, 1] == 1025 and b2[0] == 5120 and W3[0, 0] == 5184 and b3[2] == 5378
    np.testing.assert_array_equal(mlp.pack(W1, b1, W2, b2, W3, b3), p)


def test_gelu_identities_and_derivative():
    z = np.linspace(-6, 6, 241)
    g = mlp.gelu(z)
    # odd part of GELU is z/2: g(z) - g(-z) = z
    np.testing.assert_allclose(g - mlp.gelu(-z), z, atol=1e-15)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(mlp.gelu(np.array([30.0, -30.0])), [30.0, 0.0], atol=1e-12)
    # derivative against central differences
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, atol=1e-8)
    # the tanh form stays within 1e-3 of z * Phi(z) (exact GELU)
    from scipy.special import erf
    exact = 0.5 * z * (1 + erf(z / np.sqrt(2)))
    assert np.abs(g - exact).max() < 1e-3


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = _rand_params(4)
    X = rng.standard_normal((7, 15))
    T = rng.standard_normal((7, 3))
    L, g = mlp.loss_and_grad(p, X, T)
    idx = rng.choice(mlp.N_PARAMS, 300, replace=False)
    idx = np.concatenate([idx, [0, 959, 960, 1023, 1024, 5119, 5120, 5183, 5184, 5375, 5376, 5378]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS); e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, T)[0] - mlp.loss_and_grad(p - e, X, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_network_reduces_to_hand_computation():
    # W1 = 0, W2 = 0: the hidden layers are constant gelu(b1) and gelu(b2)
    W1 = np.zeros((64, 15)); W2 = np.zeros((64, 64))
    b1 = np.linspace(-1, 1, 64); b2 = np.linspace(2, -2, 64)
    W3 = np.zeros((3, 64)); W3[0, 5] = 2.0; W3[2, 63] = -1.0
    b3 = np.array([0.5, -0.25, 1.0])
    p = mlp.pack(W1, b1, W2, b2, W3, b3)
    Y, _ = mlp.forward(p, np.random.default_rng(0).standard_normal((4, 15)))
    g = lambda z: 0.5 * z * (1 + np.tanh(np.sqrt(2 / np.pi) * (z + 0.044715 * z ** 3)))
    expect = np.array([0.5 + 2.0 * g(b2[5]), -0.25, 1.0 - g(b2[63])])
    np.testing.assert_allclose(Y, np.tile(expect, (4, 1)), rtol=1e-15, atol=1e-15)


def test_adam_first_step_closed_form():
    # after one step the bias-corrected moments are g and g^2, so the update is -lr g / (|g| + eps)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(50); g = rng.standard_normal(50) * 1e-3
    w1, m, v = mlp.adam_step(w, np.zeros(50), np.zeros(50), g, 1, lr=0.01)
    np.testing.assert_allclose(w1 - w, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)
    # constant gradient: the bias-corrected moments stay g and g^2 at every step
    w2, m2, v2 = mlp.adam_step(w1, m, v, g, 2, lr=0.01)
    np.testing.assert_allclose(w2 - w1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-10)


@pytest.mark.parametrize("x,expect", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                      # halfway, ties to the even mantissa
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),      # halfway, ties to even (upwards)
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),
    (-3.140625, -3.140625),                      # exactly representable
    (0.1, 0.10009765625),
])
def test_bf16_rounding(x, expect):
    assert mlp.bf16_round(np.array([x]))[0] == expect


def test_feature_layout():
    rng = np.random.default_rng(9)
    us = [rng.standard_normal(12) for _ in range(4)]
    f = rng.standard_normal(12)
    X = mlp.features(us, f, 2.0, 0.5, 4.0)
    assert X.shape == (4, 15)
    node = 2
    np.testing.assert_array_equal(X[node, 0:3], us[0][6:9] / 2.0)
    np.testing.assert_allclose(X[node, 3:6], (us[0][6:9] - us[1][6:9]) / 0.5, rtol=1e-15)
    np.testing.assert_allclose(X[node, 9:12], (us[2][6:9] - us[3][6:9]) / 0.5, rtol=1e-15)
    np.testing.assert_array_equal(X[node, 12:15], f[6:9] / 4.0)
    # the encoding is invertible: the four displacements come back
    d = X[:, 3:12].reshape(4, 3, 3) * 0.5
    u1 = X[:, 0:3] * 2.0
    np.testing.assert_allclose(u1 - d[:, 0] - d[:, 1] - d[:, 2], us[3].reshape(4, 3), atol=1e-14)
