"""Pins for the FP64 cost-model network (CPU only): central finite
differences for the backward pass, closed forms for Adam's first step."""
import numpy as np

from oracle import mlp


def test_param_count():
    assert mlp.N_PARAMS == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2 == 5378


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init(1)
    theta[mlp.N_PARAMS - 2:] = rng.normal(0, 0.1, 2)
    x = rng.normal(0, 1, (32, 16))
    t = rng.normal(0, 1, (32, 2))
    g = mlp.backward(theta, x, t)
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False)
    fd = mlp.finite_diff(theta, x, t, idx, h=1e-6)
    np.testing.assert_allclose(g[idx], fd, rtol=1e-5, atol=1e-8)


def test_forward_closed_form_zero_weights():
    theta = np.zeros(mlp.N_PARAMS)
    p = mlp.unpack(theta)
    p["b3"][:] = [1.5, -2.0]
    y, _ = mlp.forward(mlp.pack(p), np.ones((3, 16)))
    assert np.array_equal(y, np.tile([1.5, -2.0], (3, 1)))


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(2)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = mlp.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    np.testing.assert_allclose(new, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
