"""Reduced reweighting (test infrastructure only).

The paper's code (ii) (Sec. 3.3, eq. reweighting2, and Sec. 4.1-4.2): once the
multicanonical weight w(E) is known, the density of states is inversely
proportional to it, D(E) ~ 1/w(E), so any average of a function of the
energy at inverse temperature beta follows from the weight alone.  The paper
computes E, C, F and S this way, in logarithms.

Readings (the same ones the GPU path takes):

* The sum runs over the reachable levels m (E = 4m - 2N; levels 1 and N-1 do
  not exist), each with the weight of its bin: ln D(m) = -ln w[m >> bs] + c.
* c makes sum_m D(m) = 2^N (every configuration counted once), which fixes
  the additive constant that F and S need and that the weight leaves free.
* E = <H>, C = beta^2 (<H^2> - <H>^2), F = -ln Z / beta, S = beta (E - F), as
  the paper defines them (totals, not per site); beta > 0.

Only the test-suite may import this module.
"""
import numpy as np


def reachable_levels(L):
    N = L * L
    m = np.arange(N + 1)
    return m[(m != 1) & (m != N - 1)]


def _logsumexp(a):
    amax = np.max(a)
    return amax + np.log(np.sum(np.exp(a - amax)))


def thermo(lnW, L, bin_shift, betas):
    """E, C, F, S at each beta, from ln w per bin; returns four fp64 arrays."""
    lnW = np.asarray(lnW, dtype=np.float64)
    N = L * L
    assert lnW.size == (N >> bin_shift) + 1
    m = reachable_levels(L)
    E = (4 * m - 2 * N).astype(np.float64)
    lnD = -lnW[m >> bin_shift]
    lnD = lnD + (N * np.log(2.0) - _logsumexp(lnD))
    out = np.zeros((4, len(betas)))
    for k, beta in enumerate(betas):
        beta = float(beta)
        assert beta > 0
        a = lnD - beta * E
        lnZ = _logsumexp(a)
        p = np.exp(a - lnZ)  # Boltzmann probabilities of the levels
        e_mean = np.sum(p * E)
        c = beta * beta * np.sum(p * (E - e_mean) ** 2)
        f = -lnZ / beta
        out[:, k] = (e_mean, c, f, beta * (e_mean - f))
    return out[0], out[1], out[2], out[3]
