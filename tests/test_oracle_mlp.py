"""Pins of the FP64 surrogate-MLP reference: its gradient against central
finite differences of its loss, and its forward pass against a hand-computed
tiny network."""
import numpy as np

from oracle import mlp


def test_param_count():
    assert mlp.N_PARAMS == 19713


def test_gradient_matches_finite_differences():
    rs = np.random.default_rng(0)
    theta = rs.normal(0, 0.2, mlp.N_PARAMS)
    X = rs.normal(0, 1, (37, mlp.N_IN))
    t = rs.normal(0, 1, 37)
    g = mlp.gradient(theta, X, t)
    idx = rs.choice(mlp.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [mlp.N_PARAMS - 1, 0, mlp.N_IN * mlp.N_HID + 5]])   # b3, W1[0,0], b1[5]
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (mlp.loss(tp, X, t) - mlp.loss(tm, X, t)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_hand_computed():
    # one active hidden path: W1[0,0] = 2, b1 = 0; W2[0,0] = 3; w3[0] = 0.5; b3 = 0.25
    p = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    p["W1"][0, 0] = 2.0
    p["W2"][0, 0] = 3.0
    p["w3"][0] = 0.5
    p["b3"][0] = 0.25
    theta = mlp.pack(p)
    X = np.zeros((2, mlp.N_IN))
    X[0, 0] = 1.5     # relu(3) -> relu(9) -> 4.5 + 0.25
    X[1, 0] = -1.0    # relu(-2) = 0 -> 0.25
    y, _ = mlp.forward(theta, X)
    assert np.allclose(y, [4.75, 0.25], rtol=0, atol=0)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5e-3], np.float32)
    r = mlp.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -6   # tie to even
    assert abs(r[4] - (-2.5e-3)) < 2.5e-3 * 2 ** -8


def test_rounded_gradient_is_the_exact_one_with_identity_rounding():
    """The rounding points of the mixed-precision gradient are parameters of
    the same backpropagation: with the identity it is the exact gradient
    (pinned above by finite differences), and with BF16 rounding it stays
    within the relative error that 8-bit significands allow."""
    rs = np.random.default_rng(3)
    theta = rs.normal(0, 0.2, mlp.N_PARAMS)
    X = rs.normal(0, 1, (41, mlp.N_IN))
    t = rs.normal(0, 1, 41)
    g = mlp.gradient(theta, X, t)
    np.testing.assert_array_equal(mlp.gradient(theta, X, t, rnd=lambda a: a), g)
    gb = mlp.gradient(theta, X, t, rnd=mlp.bf16)
    assert 0 < np.linalg.norm(gb - g) <= 0.1 * np.linalg.norm(g)      # errors compound over two layers
    yb, _ = mlp.forward(theta, X, rnd=mlp.bf16)
    y, _ = mlp.forward(theta, X)
    assert 0 < np.abs(yb - y).max() <= 2.0 ** -6 * np.abs(y).max()
    assert mlp.loss(theta, X, t, rnd=mlp.bf16) != mlp.loss(theta, X, t)
