"""Pins of the cost-model network's CPU oracle (oracle/mlp.py) against
finite differences and closed forms."""
import numpy as np
import pytest

from oracle import mlp

DIMS = [4, 6, 5, 7, 3]


def rand_params(seed, dims=DIMS):
    g = np.random.default_rng(seed)
    return g.normal(0, 0.7, mlp.n_params(dims))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    g = np.random.default_rng(100 + seed)
    p = rand_params(seed)
    X = g.normal(size=(9, DIMS[0]))
    T = g.normal(size=(9, DIMS[-1]))
    loss, grad = mlp.loss_grad(p, DIMS, X, T)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.mse(mlp.forward(p + e, DIMS, X)[-1], T) - mlp.mse(mlp.forward(p - e, DIMS, X)[-1], T)) / (2 * h)
    # ReLU kinks make a few entries non-differentiable at measure-zero points;
    # random data keeps all pre-activations away from 0 by far more than h.
    np.testing.assert_allclose(grad, fd, rtol=1e-5, atol=1e-8)
    assert loss == pytest.approx(mlp.mse(mlp.forward(p, DIMS, X)[-1], T))


def test_forward_identity_network_passes_positive_inputs():
    dims = [3, 3, 3, 3, 3]
    layers = [(np.eye(3), np.zeros(3)) for _ in range(4)]
    p = mlp.pack(layers)
    X = np.array([[1.0, 2.0, 3.0], [0.5, -1.0, 4.0]])
    Y = mlp.forward(p, dims, X)[-1]
    np.testing.assert_array_equal(Y[0], X[0])
    np.testing.assert_array_equal(Y[1], [0.5, 0.0, 4.0])  # the negative is cut by the first ReLU


def test_bias_only_output_layer_gradient_is_mean_residual():
    """With all weights zero, the output is the last bias and dL/db_last is
    2 * mean over rows of (b - t) / outputs."""
    dims = [2, 3, 3, 3, 2]
    p = np.zeros(mlp.n_params(dims))
    b = np.array([0.3, -0.2])
    p[-2:] = b
    T = np.array([[1.0, 1.0], [0.0, -1.0], [2.0, 0.5]])
    loss, grad = mlp.loss_grad(p, dims, np.ones((3, 2)), T)
    np.testing.assert_allclose(grad[-2:], 2 * (b - T).sum(axis=0) / T.size)
    assert loss == pytest.approx(np.mean((b - T) ** 2))


def test_first_adam_step_is_lr_times_sign():
    g = np.array([0.5, -2.0, 1e-3, -1e-4])
    p, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-3)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_bias_correction_second_step():
    g1, g2 = 0.4, -0.2
    p, m, v = mlp.adam_step(np.zeros(1), np.array([g1]), np.zeros(1), np.zeros(1), 1, lr=0.1)
    p, m, v = mlp.adam_step(p, np.array([g2]), m, v, 2, lr=0.1)
    m2 = 0.9 * 0.1 * g1 + 0.1 * g2
    v2 = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    step2 = 0.1 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    np.testing.assert_allclose(p, [-0.1 * 1.0 - step2], rtol=1e-6)
