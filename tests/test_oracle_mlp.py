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


def _silu_net():
    """A sparse non-zero network whose outputs have closed forms: the
    logistic function is 3/4 at ln 3 and 1/4 at -ln 3, so silu(ln 3) =
    (3/4) ln 3 and silu(-ln 3) = -(1/4) ln 3."""
    L3 = np.log(3.0)
    p = mlp.unpack(np.zeros(mlp.N_PARAMS))
    # layer 1: unit 5 reads feature 2 plus its bias; unit 7 reads feature 0
    p["W1"][5, 2] = L3 - 1.0
    p["b1"][5] = 1.0
    p["W1"][7, 0] = -L3
    # layer 2 (square, so a transposed weight would not fail on shape):
    # unit 3 reads hidden unit 5, unit 9 reads hidden unit 7 plus its bias
    p["W2"][3, 5] = 4.0 / 3.0
    p["W2"][9, 7] = -4.0 * (L3 - 0.5) / L3
    p["b2"][9] = 0.5
    # output layer
    p["W3"][0, 3] = 2.0
    p["W3"][1, 9] = -1.0
    p["b3"][:] = [0.5, 0.25]
    return mlp.pack(p), L3


def test_forward_closed_form_silu_network():
    theta, L3 = _silu_net()
    x = np.zeros((2, 16))
    x[:, 0] = 1.0
    x[:, 2] = 1.0
    y, (_, z1, h1, z2, h2) = mlp.forward(theta, x)
    # hidden values: z1[5] = ln 3, z1[7] = -ln 3; z2[3] = z2[9] = ln 3
    np.testing.assert_allclose(h1[0, 5], 0.75 * L3, rtol=1e-14)
    np.testing.assert_allclose(h1[0, 7], -0.25 * L3, rtol=1e-14)
    np.testing.assert_allclose(h2[0, [3, 9]], [0.75 * L3, 0.75 * L3], rtol=1e-14)
    # silu(0) = 0: every other unit is silent
    assert np.count_nonzero(h1[0]) == 2 and np.count_nonzero(h2[0]) == 2
    # outputs: y0 = 2 * (3/4) ln 3 + 1/2, y1 = -(3/4) ln 3 + 1/4
    np.testing.assert_allclose(y[0], [1.5 * L3 + 0.5, -0.75 * L3 + 0.25], rtol=1e-14)
    np.testing.assert_array_equal(y[0], y[1])
    # the loss of a closed-form target
    t = np.array([[0.5, 0.25], [0.5, 0.25]])
    np.testing.assert_allclose(mlp.loss(theta, x, t),
                               0.5 * ((1.5 * L3) ** 2 + (0.75 * L3) ** 2), rtol=1e-13)


def test_forward_silu_limits():
    """silu(z) -> z for large z and -> 0 for very negative z."""
    p = mlp.unpack(np.zeros(mlp.N_PARAMS))
    p["W1"][0, 0] = 1.0
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = 1.0
    theta = mlp.pack(p)
    x = np.zeros((2, 16))
    x[0, 0] = 40.0      # silu(40) = 40 / (1 + e^-40) = 40 to double precision
    x[1, 0] = -40.0     # silu(-40) ~ -40 e^-40 ~ -1.7e-16
    y, _ = mlp.forward(theta, x)
    assert y[0, 0] == 40.0
    assert abs(y[1, 0]) < 1e-15 and y[0, 1] == 0.0


def test_backward_closed_form_silu_network():
    """Gradient of the closed-form network in the last layer: dL/dW3[o, j] =
    mean over the batch of (y_o - t_o) h2_j; with identical rows it is the
    single row's product."""
    theta, L3 = _silu_net()
    x = np.zeros((2, 16))
    x[:, 0] = 1.0
    x[:, 2] = 1.0
    t = np.zeros((2, 2))
    g = mlp.unpack(mlp.backward(theta, x, t))
    y0, y1 = 1.5 * L3 + 0.5, -0.75 * L3 + 0.25
    np.testing.assert_allclose(g["W3"][0, 3], y0 * 0.75 * L3, rtol=1e-13)
    np.testing.assert_allclose(g["W3"][1, 9], y1 * 0.75 * L3, rtol=1e-13)
    np.testing.assert_allclose(g["b3"], [y0, y1], rtol=1e-13)
    # silu'(z) = s (1 + z (1 - s)); at ln 3: 3/4 (1 + ln3 / 4)
    ds = 0.75 * (1 + L3 / 4)
    np.testing.assert_allclose(g["b2"][3], y0 * 2.0 * ds, rtol=1e-13)
