"""GPU parity of the reduced reweighting (mc_thermo, code (ii)) against the
oracle, from exact and from sampled weights, at the smallest and largest
lattices; argument errors.

Tolerances: each Boltzmann factor is exp(a_m - max a) with
a_m = ln D(m) - beta E_m, a difference of numbers as large as
A = N ln 2 + 2 beta N + max |ln w|; the two sides round it differently (the
normalisation enters at a different point, exp and log come from different
libraries), so each factor carries a relative error of order eps * A
(5e-11 at L = 256, beta = 3).  E, F and S then agree to 1e-9 relative, and C,
a variance, to 1e-7 relative (1e-9 N absolute near its zeros).
"""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

from paper_0812_2964_amd import exact as X  # noqa: E402
from oracle.thermo import thermo as o_thermo  # noqa: E402

pytestmark = pytest.mark.gpu

BETAS = np.concatenate([np.linspace(0.02, 1.0, 50), [1.5, 2.0, 3.0]])
# Largest |E - E_exact| / N after the recursion below; the run is deterministic
# (fixed seeds) and measured 0.0013 on the MI355X, so 0.005 leaves a margin
# while still catching a wrong weight, level range or normalisation.
TOL_E_RECURSION = 0.005


def _mc():
    import paper_0812_2964_amd as mc

    return mc


def _check(g, o, N):
    e, c, f, s = g
    oe, oc, of, os_ = o
    assert np.allclose(e, oe, rtol=1e-9, atol=1e-9 * N)
    assert np.allclose(f, of, rtol=1e-9, atol=1e-9 * N)
    assert np.allclose(s, os_, rtol=1e-9, atol=1e-9 * N)
    assert np.allclose(c, oc, rtol=1e-7, atol=1e-9 * N)


def test_exact_weight_L8():
    mc = _mc()
    L, N = 8, 64
    gd = X.transfer_dos(L).astype(np.float64)
    w = np.zeros(N + 1)
    w[gd > 0] = -np.log(gd[gd > 0])
    ctx = mc.Context([(L, 4, 1, 0)])
    ctx.init_weights(w)
    _check(ctx.thermo(BETAS), o_thermo(w, L, 0, BETAS), N)
    ctx.close()


@pytest.mark.parametrize("L", [32, 256])
def test_binned_weights_small_and_largest(L):
    mc = _mc()
    N = L * L
    nb = (N >> 1) + 1
    if L == 32:
        w = np.load(os.path.join(HERE, "golden", "lnW_L32_prior.npy"))
    else:
        rng = np.random.default_rng(9)
        x = (np.arange(nb) - nb / 2) / nb
        w = -0.6 * N * x * x + np.cumsum(rng.normal(0, 0.05, nb))
    ctx = mc.Context([(L, 2, 1, 1)])
    ctx.init_weights(w)
    _check(ctx.thermo(BETAS), o_thermo(w, L, 1, BETAS), N)
    ctx.close()


def test_after_recursion_and_against_kaufman():
    """A recursion at L = 8 with one bin per level (20 graph-captured
    iterations of 64 chains x 10^4 sweeps from ln w = 0): the weight it reaches
    gives the oracle's numbers on the GPU, and E agrees with Kaufman's exact
    finite-lattice energy within the statistical error of that weight.  (With
    width-8 bins the reduced formula gives both levels of a bin the same
    density, a bias of up to 6 % of N at L = 8 even with exact bin weights.)"""
    import torch

    mc = _mc()
    L, P, M = 8, 64, 10000
    N = L * L
    ctx = mc.Context([(L, P, 1, 0)])
    tr, h, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
    g = ctx.graph(M, 20, [tr], [h], [cut])
    g.launch()
    torch.cuda.synchronize()
    g.close()
    w = ctx.weights()
    betas = np.array([0.1, 0.3, 0.4407, 0.6, 1.0])
    res = ctx.thermo(betas)
    _check(res, o_thermo(w, L, 0, betas), N)
    dev = [abs(res[0][k] - X.mean_energy_exact(L, b)) / N for k, b in enumerate(betas)]
    print("E deviation from Kaufman / N:", ["%.4f" % d for d in dev])
    assert max(dev) < TOL_E_RECURSION
    ctx.close()


def test_argument_errors():
    mc = _mc()
    ctx = mc.Context([(8, 2, 1, 1)])
    for bad in ([0.0], [-1.0], [float("nan")], [float("inf")]):
        with pytest.raises(mc.MCError):
            ctx.thermo(bad)
    with pytest.raises(mc.MCError):
        ctx.thermo([])
    ctx.close()
