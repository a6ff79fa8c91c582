"""Pins of the oracle's reduced reweighting (code (ii), eq. reweighting2).

Given the exact multicanonical weight ln w = -ln g, the reweighting must give
the exact thermodynamics of the finite periodic lattice:

* L = 4: against a direct sum over all 2^16 spin configurations (no density of
  states involved);
* L = 8: against Kaufman's closed form of ln Z and its derivatives in beta;
* invariants: a constant added to ln w changes nothing; width-2 bins equal the
  per-level weights they expand to; the low- and high-temperature limits.
"""
import os
import sys

import mpmath
import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

from paper_0812_2964_amd import exact as X  # noqa: E402
from oracle.thermo import thermo  # noqa: E402

BETAS = [0.05, 0.2, 0.35, 0.4407, 0.5, 0.7, 1.0]


def _exact_weight(g):
    g = np.asarray(g, dtype=np.float64)
    w = np.zeros(g.size)
    w[g > 0] = -np.log(g[g > 0])
    return w


def _all_energies_L4():
    """Energy of every configuration of the 4 x 4 torus, one spin per bit."""
    L, N = 4, 16
    s = np.arange(1 << N, dtype=np.int64)
    spin = np.stack([((s >> j) & 1) * 2 - 1 for j in range(N)], axis=1)
    E = np.zeros(1 << N, dtype=np.int64)
    for y in range(L):
        for x in range(L):
            j = y * L + x
            E -= spin[:, j] * spin[:, y * L + (x + 1) % L]
            E -= spin[:, j] * spin[:, ((y + 1) % L) * L + x]
    return E.astype(np.float64)


def test_L4_against_every_configuration():
    g = X.brute_force_dos(4)
    E_s = _all_energies_L4()
    e, c, f, s = thermo(_exact_weight(g), 4, 0, BETAS)
    for k, beta in enumerate(BETAS):
        a = -beta * E_s
        amax = a.max()
        wts = np.exp(a - amax)
        Z = wts.sum()
        lnZ = amax + np.log(Z)
        e_ref = (wts * E_s).sum() / Z
        c_ref = beta * beta * ((wts * E_s * E_s).sum() / Z - e_ref * e_ref)
        f_ref = -lnZ / beta
        assert e[k] == pytest.approx(e_ref, rel=1e-11, abs=1e-11)
        assert c[k] == pytest.approx(c_ref, rel=1e-9, abs=1e-11)
        assert f[k] == pytest.approx(f_ref, rel=1e-12)
        assert s[k] == pytest.approx(beta * (e_ref - f_ref), rel=1e-10, abs=1e-10)


def test_L8_against_kaufman():
    L = 8
    g = X.transfer_dos(L)
    e, c, f, s = thermo(_exact_weight(g), L, 0, BETAS)
    with mpmath.workprec(300):
        h = mpmath.mpf("1e-30")
        for k, beta in enumerate(BETAS):
            b = mpmath.mpf(beta)
            lz0 = X.kaufman_lnZ(L, b)
            lzp, lzm = X.kaufman_lnZ(L, b + h), X.kaufman_lnZ(L, b - h)
            e_ref = float(-(lzp - lzm) / (2 * h))
            c_ref = float(b * b * (lzp - 2 * lz0 + lzm) / (h * h))
            f_ref = float(-lz0 / b)
            s_ref = float(b * (-(lzp - lzm) / (2 * h)) + lz0)
            assert f[k] == pytest.approx(f_ref, rel=1e-12)
            assert e[k] == pytest.approx(e_ref, rel=1e-10)
            assert c[k] == pytest.approx(c_ref, rel=1e-8)
            assert s[k] == pytest.approx(s_ref, rel=1e-10)


def test_constant_shift_and_bins():
    rng = np.random.default_rng(3)
    L, N = 8, 64
    w_bins = rng.normal(0, 3, (N >> 1) + 1)
    a = np.array(thermo(w_bins, L, 1, BETAS))
    b = np.array(thermo(w_bins + 17.25, L, 1, BETAS))
    assert np.allclose(a, b, rtol=1e-12, atol=1e-10)
    # width-2 bins are the per-level weight that gives both levels the bin's value
    w_levels = w_bins[np.arange(N + 1) >> 1]
    c = np.array(thermo(w_levels, L, 0, BETAS))
    assert np.allclose(a, c, rtol=1e-12, atol=1e-10)


def test_temperature_limits():
    L, N = 8, 64
    g = X.transfer_dos(L)
    w = _exact_weight(g)
    e, c, f, s = thermo(w, L, 0, [30.0])
    assert e[0] == pytest.approx(-2 * N, rel=1e-12)  # ground state
    assert s[0] == pytest.approx(np.log(2.0), abs=1e-9)  # two ground states
    assert c[0] < 1e-9
    e, c, f, s = thermo(w, L, 0, [1e-7])
    assert s[0] == pytest.approx(N * np.log(2.0), abs=1e-6)  # all 2^N configurations
    assert abs(e[0]) < 1e-3
