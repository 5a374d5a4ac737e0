"""FP64 reference of the learned step proposer (MLP 8 -> 64 -> 64 -> 1, ReLU).

TEST INFRASTRUCTURE ONLY (the GPU kernels are checked against it).

Parameter vector (4801): W1[64][8] b1[64] W2[64][64] b2[64] w3[64] b3.
Normalisation (18): feature means[8], feature std devs[8], target mean, std.
Loss: mean squared error between the network output and the normalised
target, L = (1/B) sum_s (y_s - (t_s - t_mean) / t_std)^2.
"""
import numpy as np

IN, HID = 8, 64
W1, B1 = 0, HID * IN
W2 = B1 + HID
B2 = W2 + HID * HID
W3 = B2 + HID
B3 = W3 + HID
NPARAMS = B3 + 1
assert NPARAMS == 4801


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[W1:B1].reshape(HID, IN), p[B1:W2], p[W2:B2].reshape(HID, HID), p[B2:W3], p[W3:B3], p[B3])


def normalise(x, t, norm):
    norm = np.asarray(norm, dtype=np.float64)
    xn = (np.asarray(x, np.float64) - norm[:IN]) / norm[IN:2 * IN]
    tn = None if t is None else (np.asarray(t, np.float64) - norm[2 * IN]) / norm[2 * IN + 1]
    return xn, tn


def forward(p, xn):
    """Network output on normalised inputs, with the hidden activations."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    a1 = xn @ w1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ w2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ w3 + b3
    return y, (a1, h1, a2, h2)


def predict(p, norm, x):
    """De-normalised prediction (natural log of the step) for raw features."""
    xn, _ = normalise(x, None, norm)
    y, _ = forward(p, xn)
    norm = np.asarray(norm, np.float64)
    return y * norm[2 * IN + 1] + norm[2 * IN]


def loss(p, norm, x, t):
    xn, tn = normalise(x, t, norm)
    y, _ = forward(p, xn)
    return np.mean((y - tn) ** 2)


def gradient(p, norm, x, t):
    """Analytic gradient of loss() by the chain rule (back-propagation)."""
    xn, tn = normalise(x, t, norm)
    w1, b1, w2, b2, w3, b3 = unpack(p)
    y, (a1, h1, a2, h2) = forward(p, xn)
    B = len(y)
    dy = 2.0 * (y - tn) / B
    g = np.zeros(NPARAMS)
    g[W3:B3] = h2.T @ dy
    g[B3] = dy.sum()
    d2 = np.outer(dy, w3) * (a2 > 0)
    g[W2:B2] = (d2.T @ h1).ravel()
    g[B2:W3] = d2.sum(axis=0)
    d1 = (d2 @ w2) * (a1 > 0)
    g[W1:B1] = (d1.T @ xn).ravel()
    g[B1:W2] = d1.sum(axis=0)
    return g
