"""FP64 reference of the surrogate MLP (test infrastructure).

The surrogate that pre-screens offspring is a per-tetrahedron multilayer
perceptron 23 -> 128 -> 128 -> 1 with ReLU activations and mean squared
error loss.  This module evaluates it and its exact gradient with plain NumPy
in FP64 so that the GPU kernels' forward pass and backward pass can be
checked against it.  The surrogate is this build's own addition (no
counterpart in the paper), so there is no passage of the paper to cite; the
mathematics is the textbook chain rule for a dense network.

Parameter order (a flat vector of 19,713 values), shared with the library's
parameter buffer:
    W1 [128][23], b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1]
where layer k computes h_k = relu(W_k h_{k-1} + b_k) and the output is
y = w3 . h_2 + b3.
"""
import numpy as np

N_IN, N_HID = 23, 128
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("w3", (N_HID,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SHAPES])


def _keep(a):
    return a


def forward(theta, X, rnd=None):
    """Predictions y [n] for inputs X [n][23], and the activations.

    ``rnd`` (default: none) rounds at the points where a matrix-core
    implementation stores operands in a narrow type: the inputs, W1, W2 and
    the layer-1 activations h1; biases, z2, h2, w3 and the output stay
    unrounded."""
    r = _keep if rnd is None else rnd
    p = unpack(theta)
    X = r(np.asarray(X, np.float64))
    z1 = X @ r(p["W1"]).T + p["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ r(p["W2"]).T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (X, z1, h1, z2, h2)


def loss(theta, X, t, rnd=None):
    y, _ = forward(theta, X, rnd)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def gradient(theta, X, t, rnd=None):
    """Gradient of the mean squared error with respect to theta (exact
    backpropagation when ``rnd`` is None).

    With ``rnd``, the forward pass rounds as in ``forward`` and the backward
    pass rounds the two back-propagated activations that a matrix-core
    implementation feeds to its products, dz2 (before dh1 = dz2 W2 and
    dW2 = dz2^T h1) and dz1 (before dW1 = dz1^T X); the bias and output-layer
    gradients use the unrounded dz2 and dz1, and the ReLU derivative of layer
    1 is taken from the rounded h1 (h1 > 0 exactly when z1 > 0 for any
    rounding that keeps signs and zeros)."""
    r = _keep if rnd is None else rnd
    p = unpack(theta)
    y, (X, z1, h1, z2, h2) = forward(theta, X, rnd)
    n = X.shape[0]
    dy = 2.0 * (y - np.asarray(t, np.float64)) / n
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["w3"]) * (z2 > 0)
    g["b2"] = dz2.sum(axis=0)
    dz2 = r(dz2)
    g["W2"] = dz2.T @ h1
    dz1 = (dz2 @ r(p["W2"])) * (h1 > 0)
    g["b1"] = dz1.sum(axis=0)
    g["W1"] = r(dz1).T @ X
    return pack(g)


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) and return as FP64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32) << 16
    return r.view(np.float32).astype(np.float64)
