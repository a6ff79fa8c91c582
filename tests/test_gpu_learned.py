"""The learned initial weight on the GPU: fp32 forward, gradient and Adam steps
against the fp64 oracle, training targets and predicted weights against their
definitions, and the gain over the plain recursion from ln w = 0."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def _mc():
    import paper_0812_2964_amd as mc

    return mc


def _problem(n=600, seed=0):
    rng = np.random.default_rng(seed)
    params = rng.normal(0, 0.3, O.mlp_n_params()).astype(np.float32)
    x = np.column_stack([1.0 / rng.choice([8, 12, 16, 24, 32], n), rng.uniform(-2.0, 2.0, n)]).astype(np.float32)
    t = rng.uniform(0.0, 0.7, n).astype(np.float32)
    w = rng.uniform(0.5, 2.0, n).astype(np.float32)
    return params, x, t, w


def test_forward_and_gradient_match_fp64_oracle():
    import torch

    mc = _mc()
    params, x, t, w = _problem()
    net = mc.MLP(params=params)
    xd, td, wd = (torch.from_numpy(a).cuda() for a in (x, t, w))
    y = net.forward(xd).cpu().numpy()
    y64 = O.mlp_forward(params.astype(np.float64), x.astype(np.float64))
    assert np.abs(y - y64).max() <= 2e-5 * max(1.0, np.abs(y64).max())
    loss, g = net.loss_grad(xd, td, wd)
    l64, g64 = O.mlp_loss_grad(params.astype(np.float64), x.astype(np.float64), t.astype(np.float64),
                               w.astype(np.float64))
    assert abs(float(loss.item()) - l64) <= 1e-4 * l64
    g = g.cpu().numpy()
    assert np.abs(g - g64).max() <= 1e-3 * np.abs(g64).max()


@pytest.mark.parametrize("n", [1, 63, 65, 10917])
def test_gradient_at_ragged_and_large_sample_counts(n):
    """The gradient's sample loop (one wave per parameter, 64 lanes over the
    samples) at one sample, either side of a wave's width, and the sample
    count of training on L in {8, 16, 32, 64, 128} (10917 bins)."""
    import torch

    mc = _mc()
    params, x, t, w = _problem(n, seed=n)
    net = mc.MLP(params=params)
    xd, td, wd = (torch.from_numpy(a).cuda() for a in (x, t, w))
    loss, g = net.loss_grad(xd, td, wd)
    l64, g64 = O.mlp_loss_grad(params.astype(np.float64), x.astype(np.float64), t.astype(np.float64),
                               w.astype(np.float64))
    assert abs(float(loss.item()) - l64) <= 1e-4 * l64
    g = g.cpu().numpy()
    assert np.abs(g - g64).max() <= 1e-3 * np.abs(g64).max()


def test_adam_steps_match_reference():
    import torch

    mc = _mc()
    params, x, t, w = _problem(200, seed=3)
    net = mc.MLP(params=params)
    xd, td, wd = (torch.from_numpy(a).cuda() for a in (x, t, w))
    net.train(xd, td, wd, steps=5, lr=1e-3)
    # Adam (beta 0.9 / 0.999, eps 1e-8) on the fp64 oracle's gradients
    p = params.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for k in range(1, 6):
        _, g = O.mlp_loss_grad(p, x.astype(np.float64), t.astype(np.float64), w.astype(np.float64))
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        p = p - 1e-3 * (m / (1 - 0.9**k)) / (np.sqrt(v / (1 - 0.999**k)) + 1e-8)
    got = net.params.cpu().numpy().astype(np.float64)
    # each step moves a parameter by at most ~lr; compare the moves
    assert np.abs((got - params) - (p - params)).max() <= 2e-4
    assert net.step.value == 5


def test_targets_and_prediction_match_definitions():
    mc = _mc()
    L, bs = 12, 1
    N = L * L
    nb = (N >> bs) + 1
    rng = np.random.default_rng(5)
    lnW = -np.cumsum(rng.uniform(-1, 1, nb))  # any finite weight
    x, t = mc.mlp_targets(lnW, L, bs)
    x, t = x.cpu().numpy(), t.cpu().numpy()
    c = N * np.log(2.0) - np.logaddexp.reduce(-lnW)
    assert np.allclose(t, (-lnW + c) / N, rtol=0, atol=2e-6)
    e = (4.0 * (2 * np.arange(nb) + 0.5) - 2 * N) / N
    assert np.allclose(x[:, 0], np.float32(1.0 / L)) and np.allclose(x[:, 1], e.astype(np.float32))
    # sum over bins of exp(N t) = 2^N
    assert abs(np.logaddexp.reduce(N * t.astype(np.float64)) - N * np.log(2.0)) < 1e-3
    params, _, _, _ = _problem(10, seed=9)
    net = mc.MLP(params=params)
    pw = net.predict_weights(L, bs)
    want = -N * O.mlp_forward(params.astype(np.float64), x.astype(np.float64))
    assert np.abs(pw - want).max() <= 3e-5 * N


def test_learned_weight_beats_plain_recursion():
    """Trained on the converged weights of L = 8, 12, 16, the network's
    proposal for L = 24 reaches a flat histogram in far fewer iterations than
    the recursion from ln w = 0 (Sec. 3.1, w^(1) = 1)."""
    from paper_0812_2964_amd.learned import Initializer, relative_spread, run_to_flat

    P, M = 512, 2000
    ini = Initializer(seed=1)
    conv = {}
    for L, cap in [(8, 40), (12, 80), (16, 120)]:
        w, flat, _ = run_to_flat(L, P, M, cap, extra=4)
        assert flat is not None, L
        conv[L] = w
        ini.add(L, w)
    loss = ini.fit(steps=4000, lr=2e-3)
    assert loss < 1e-3
    # the network reproduces its training weights up to a few nats
    for L in (8, 12, 16):
        assert relative_spread(ini.predict(L), conv[L]) < 0.05 * L * L
    _, flat0, _ = run_to_flat(24, P, M, 120)
    _, flat1, _ = run_to_flat(24, P, M, 120, lnW0=ini.predict(24))
    assert flat1 is not None
    assert flat0 is None or flat1 * 3 <= flat0
