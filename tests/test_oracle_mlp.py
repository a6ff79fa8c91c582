"""Pins of the fp64 network oracle: gradient against central differences,
forward against closed forms."""
import math

import numpy as np

import oracle as O

H = 64


def test_n_params():
    assert O.mlp_n_params() == 2 * H + H + H * H + H + H + 1 == 4417


def test_forward_closed_forms():
    n = O.mlp_n_params()
    x = np.array([[0.125, -1.5], [0.05, 0.3]])
    p = np.zeros(n)
    p[-1] = 0.7  # only the output bias
    assert np.allclose(O.mlp_forward(p, x), 0.7, rtol=0, atol=0)
    # W2 = 0: layer 2 sees only its biases; y = b3 + sum_j W3_j tanh(b2_j)
    rng = np.random.default_rng(1)
    p = rng.normal(0, 0.5, n)
    off_w2, off_b2, off_w3 = 2 * H + H, 2 * H + H + H * H, 2 * H + H + H * H + H
    p[off_w2:off_b2] = 0.0
    want = p[-1] + sum(p[off_w3 + j] * math.tanh(p[off_b2 + j]) for j in range(H))
    assert np.allclose(O.mlp_forward(p, x), want, rtol=1e-14)
    # one hidden path: unit 0 of each layer only
    p = np.zeros(n)
    p[0], p[1], p[2 * H] = 0.5, -0.25, 0.1  # W1[0], b1[0]
    p[off_w2] = 2.0                          # W2[0][0]
    p[off_w3] = 3.0                          # W3[0]
    xx = x[0]
    want = 3.0 * math.tanh(2.0 * math.tanh(0.5 * xx[0] - 0.25 * xx[1] + 0.1))
    assert abs(O.mlp_forward(p, x[:1])[0] - want) < 1e-15


def test_gradient_against_central_differences():
    n = O.mlp_n_params()
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, n)
    x = np.column_stack([1.0 / rng.choice([8, 12, 16, 24], 40), rng.uniform(-2, 2, 40)])
    t = rng.normal(0.3, 0.2, 40)
    w = rng.uniform(0.5, 2.0, 40)
    _, g = O.mlp_loss_grad(p, x, t, w)
    idx = np.concatenate([np.arange(0, 200), rng.choice(n, 400, replace=False), [n - 1]])
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        num = (O.mlp_loss_grad(pp, x, t, w)[0] - O.mlp_loss_grad(pm, x, t, w)[0]) / (2 * h)
        assert abs(num - g[k]) <= 1e-6 * np.abs(g).max() + 1e-9, k
    # the loss is the weighted mean squared error
    y = O.mlp_forward(p, x)
    assert abs(O.mlp_loss_grad(p, x, t, w)[0] - (w * (y - t) ** 2).sum() / w.sum()) < 1e-12
