"""Pins of the oracle's Ising model and Metropolis sweeps against exact physics.

* The oracle's energy function, summed over all 2^16 states of the 4 x 4
  torus, reproduces Kaufman's exact partition function (and an independent
  brute-force count).
* The reachable levels match exact transfer-matrix densities of states.
* Sweeps with the exact multicanonical weight -ln g give a flat level
  histogram; sweeps with Boltzmann weights give the exact canonical
  distribution and the exact mean energy (Sec. 3 of the paper: the sampled
  distribution is D(E) w(E) up to normalisation).
* With ln w = 0 every move is accepted, so typewriter sweeps negate the
  lattice and the energy is constant (deterministic special case).
"""
import numpy as np
import pytest

from paper_0812_2964_amd import exact as X
import oracle as O


def test_energy_reproduces_kaufman_at_L4():
    L, N = 4, 16
    g = np.zeros(N + 1, dtype=np.int64)
    for state in range(1 << N):
        s = np.array([1 if (state >> j) & 1 else -1 for j in range(N)], dtype=np.int8)
        e = O.energy(L, s)
        assert (e + 2 * N) % 4 == 0
        g[(e + 2 * N) // 4] += 1
    assert np.array_equal(g, X.brute_force_dos(4))
    for K in (0.1, 0.3, 0.4406867935097715, 0.6, 1.0):
        assert abs(float(X.lnZ_from_dos(g, L, K) - X.kaufman_lnZ(L, K))) < 1e-12


def test_energy_single_flip_changes():
    # flipping one spin of the ground state breaks 4 bonds: dE = +8
    for L in (4, 6, 8):
        s = np.ones(L * L, dtype=np.int8)
        e0 = O.energy(L, s)
        assert e0 == -2 * L * L
        s[L + 1] = -1
        assert O.energy(L, s) == e0 + 8
        s[L + 2] = -1  # neighbouring pair: 6 broken bonds
        assert O.energy(L, s) == e0 + 12
        cb = np.array([(-1) ** (x + y) for y in range(L) for x in range(L)], dtype=np.int8)
        assert O.energy(L, cb) == 2 * L * L  # checkerboard: all bonds broken


@pytest.mark.parametrize("L", [4, 6, 8])
def test_reachable_levels_match_exact(L):
    g = X.brute_force_dos(L) if L == 4 else X.transfer_dos(L)
    for m in range(L * L + 1):
        assert O.level_reachable(L, m) == (g[m] > 0)
    # symmetry g(E) = g(-E) of the bipartite torus
    assert np.array_equal(g, g[::-1])


def test_kaufman_against_transfer_matrix_L8():
    g = X.transfer_dos(8)
    assert sum(int(v) for v in g) == 2**64
    for K in (0.2, 0.4406867935097715, 0.7):
        assert abs(float(X.lnZ_from_dos(g, 8, K) - X.kaufman_lnZ(8, K))) < 1e-12


def test_init_chain_bits():
    L, seed = 8, 1
    s = O.init_chain(L, seed, 5)
    for j in range(L * L):
        assert s[j] == (1 if O.uniform(seed, L, 1, 0, 5, j) >> 31 else -1)
    allspins = np.concatenate([O.init_chain(32, 1, c) for c in range(16)])
    assert abs((allspins == 1).mean() - 0.5) < 0.01


def test_tabulate_closed_form():
    L, bs = 4, 1
    nb = O.n_bins(L, bs)
    rng = np.random.default_rng(0)
    lnW = rng.normal(0, 3, nb)
    T = O.tabulate(L, bs, lnW)
    N = L * L
    for m in range(N + 1):
        for a in range(5):
            mt = m + a - 2
            if mt < 0 or mt > N:
                assert T[m, a] == 0
            else:
                assert T[m, a] == O.threshold(lnW[mt >> bs] - lnW[m >> bs])
        assert T[m, 2] == 0xFFFFFFFF
    T0 = O.tabulate(L, bs, np.zeros(nb))
    for m in range(N + 1):
        for a in range(5):
            if 0 <= m + a - 2 <= N:
                assert T0[m, a] == 0xFFFFFFFF


def test_lnW_zero_sweeps_are_deterministic():
    for L in (4, 8, 12):
        N = L * L
        s0 = O.init_chain(L, 1, 3)
        m0 = (O.energy(L, s0) + 2 * N) // 4
        s, m, tr, h = O.sweeps(L, 1, 1, 3, s0, m0, 0, 7, np.zeros(O.n_bins(L, 1)))
        assert np.array_equal(s, -s0)  # odd number of sweeps: negated
        assert m == m0
        assert np.all(tr == m0 - N // 2)
        assert h[m0 >> 1] == 7 and h.sum() == 7


def test_tracked_level_matches_lattice():
    L, N = 8, 64
    rng = np.random.default_rng(4)
    lnW = rng.normal(0, 2, O.n_bins(L, 1))
    s = O.init_chain(L, 1, 0)
    m = (O.energy(L, s) + 2 * N) // 4
    s, m, tr, h = O.sweeps(L, 1, 1, 0, s, m, 0, 500, lnW)
    assert (O.energy(L, s) + 2 * N) // 4 == m
    assert tr[-1] == m - N // 2
    assert h.sum() == 500
    assert np.all((tr + N // 2 != 1) & (tr + N // 2 != N - 1))  # unreachable levels never appear


def test_exact_multicanonical_weight_gives_flat_histogram():
    L, N = 4, 16
    g = X.brute_force_dos(L)
    lnW = np.where(g > 0, -np.log(np.maximum(g, 1)), 0.0)
    s = O.init_chain(L, 1, 0)
    m = (O.energy(L, s) + 2 * N) // 4
    _, _, tr, h = O.sweeps(L, 1, 0, 0, s, m, 0, 200000, lnW)
    hr = h[g > 0]
    assert np.abs(hr / hr.mean() - 1).max() < 0.04
    # level-resolved symmetry of the sampled distribution
    assert np.abs(hr / hr[::-1] - 1).max() < 0.06


@pytest.mark.parametrize("beta", [0.3, 0.6])
def test_boltzmann_weight_gives_canonical_ensemble(beta):
    L, N = 4, 16
    g = X.brute_force_dos(L)
    E = 4 * np.arange(N + 1) - 2 * N
    lnW = -beta * E  # one bin per level (bin_shift 0)
    s = O.init_chain(L, 1, 1)
    m = (O.energy(L, s) + 2 * N) // 4
    M = 200000
    _, _, tr, h = O.sweeps(L, 1, 0, 1, s, m, 0, M, lnW)
    p = g * np.exp(-beta * (E - E.min()))
    p = p / p.sum()
    big = p * M > 500
    rel = np.abs(h[big] / (p[big] * M) - 1)
    assert rel.max() < 0.05
    e_mean = (4 * (tr + N // 2) - 2 * N).mean()
    # the chain's own batch-means error bar
    eb = (4 * (tr + N // 2) - 2 * N).reshape(100, -1).mean(axis=1)
    err = eb.std(ddof=1) / np.sqrt(len(eb))
    assert abs(e_mean - X.mean_energy_exact(L, beta)) < 5 * err + 1e-9
