"""Pins of the FP64 surrogate-network oracle (oracle/mlp.py)."""
import numpy as np

import workloads
from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 34052
    assert workloads.mlp_init().shape == (34052,)


def test_silu_closed_forms():
    assert mlp.silu(0.0) == 0.0 and mlp.dsilu(0.0) == 0.5
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.dsilu(z)).max() < 1e-9
    assert np.allclose(mlp.silu(z), z / (1 + np.exp(-z)))


def test_zero_weights_give_output_bias():
    theta = np.zeros(mlp.N_PARAMS)
    p = mlp.unflatten(theta)
    p["b4"][:] = [1.5, -2.0, 0.25, 3.0]
    p["b1"][:] = 0.7  # hidden biases do not reach the output through zero W4
    y, _ = mlp.forward(mlp.flatten(p), np.random.default_rng(0).normal(size=(5, 3)))
    assert np.array_equal(y, np.tile([1.5, -2.0, 0.25, 3.0], (5, 1)))


def test_single_hidden_path_closed_form():
    # One path x0 -> unit 0 of every layer -> output 0: y = w4 silu(w3 silu(w2 silu(w1 x0)))
    theta = np.zeros(mlp.N_PARAMS)
    p = mlp.unflatten(theta)
    p["W1"][0, 0], p["W2"][0, 0], p["W3"][0, 0], p["W4"][0, 0] = 0.9, -1.3, 0.7, 2.0
    x = np.array([[0.4, 5.0, -3.0]])
    y, _ = mlp.forward(mlp.flatten(p), x)
    s = mlp.silu
    assert np.isclose(y[0, 0], 2.0 * s(0.7 * s(-1.3 * s(0.9 * 0.4))), rtol=1e-15)
    assert np.all(y[0, 1:] == 0.0)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = workloads.mlp_init(5)
    x = rng.uniform(0, 1, size=(16, 3))
    t = rng.normal(size=(16, 4))
    w = np.array([1.0, 0.5, 0.5, 0.5])
    _, g = mlp.loss_grad(theta, x, t, w)
    idx = rng.choice(mlp.N_PARAMS, size=60, replace=False)
    idx = np.concatenate([idx, [0, 383, 384, 511, 34051, 34047, 33536]])
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (mlp.loss_grad(tp, x, t, w)[0] - mlp.loss_grad(tm, x, t, w)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_adam_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2: the update is -lr g/(|g| + eps)
    rng = np.random.default_rng(4)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    th1, m, v = mlp.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    assert np.allclose(th1, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-16)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_ties_to_even():
    one = 1.0
    assert mlp.round_bf16(np.array([one]))[0] == 1.0
    assert mlp.round_bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0            # tie -> even
    assert mlp.round_bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6  # tie -> even
    assert mlp.round_bf16(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7
    assert mlp.round_bf16(np.array([-3.140625]))[0] == -3.140625
