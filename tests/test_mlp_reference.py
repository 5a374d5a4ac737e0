"""Pins of the FP64 reference MLP: the analytic gradient equals central finite
differences of the loss; closed forms for a network reduced to a line."""
import numpy as np

from oracle import mlp


def _setup(seed=0, n=40):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.NPARAMS)
    norm = np.concatenate([rng.normal(0, 1, 8), rng.uniform(0.5, 2, 8), [rng.normal(), rng.uniform(0.5, 2)]])
    x = rng.normal(0, 1, (n, 8)) * norm[8:16] + norm[:8]
    t = rng.normal(0, 1, n)
    return p, norm, x, t


def test_gradient_matches_finite_differences():
    p, norm, x, t = _setup()
    g = mlp.gradient(p, norm, x, t)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.NPARAMS, 300, replace=False), [mlp.B3, mlp.W1, mlp.B1, mlp.W3]])
    h = 1e-6
    for q in idx:
        e = np.zeros(mlp.NPARAMS)
        e[q] = h
        fd = (mlp.loss(p + e, norm, x, t) - mlp.loss(p - e, norm, x, t)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(g[q])), q


def test_linear_closed_form():
    # with W2 = identity on the positive part and positive inputs, the network
    # reduces to y = w3 . (W1 x + b1) + b3 for inputs that keep every unit active
    p = np.zeros(mlp.NPARAMS)
    W1 = np.zeros((64, 8))
    W1[0, 0] = 1.0
    W1[1, 1] = 2.0
    p[mlp.W1:mlp.B1] = W1.ravel()
    p[mlp.B1:mlp.W2] = 1.0  # keeps units active for |x| < 0.5
    p[mlp.W2:mlp.B2] = np.eye(64).ravel()
    p[mlp.W3:mlp.B3] = 0.5
    p[mlp.B3] = -3.0
    norm = np.concatenate([np.zeros(8), np.ones(8), [0.0, 1.0]])
    x = np.random.default_rng(2).uniform(-0.4, 0.4, (10, 8))
    y = mlp.predict(p, norm, x)
    assert np.allclose(y, 0.5 * (64 + x[:, 0] + 2 * x[:, 1]) - 3.0, rtol=1e-14, atol=1e-12)
