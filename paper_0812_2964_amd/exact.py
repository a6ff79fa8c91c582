"""Exact results for the periodic 2D Ising model (J = 1): the reference values
the thermodynamics of a multicanonical weight are judged by (Sec. 5 compares
with exact finite-lattice results), and pins of the test oracle.

None of this is part of the sampling method; it is independent mathematics:

* ``brute_force_dos(L)`` enumerates all 2^(L*L) configurations (L = 4 only).
* ``transfer_dos(L)`` counts configurations per energy exactly with a row
  transfer matrix (even L <= 8), integer arithmetic throughout.
* ``kaufman_lnZ(L, K)`` is Kaufman's closed form of the partition function of
  an L x L torus (B. Kaufman, Phys. Rev. 76 (1949) 1232), the finite-lattice
  result that the paper compares its thermodynamics with (Sec. 5, exact
  results of Ferdinand and Fisher, which rest on it).

Energies are expressed through the level m = (E + 2N)/4 = (number of broken
bonds)/2, so a density of states is an int64 array of length N + 1.
"""
import functools

import mpmath
import numpy as np


def _popcount(a):
    a = np.asarray(a, dtype=np.int64)
    c = np.zeros_like(a)
    while np.any(a):
        c += a & 1
        a = a >> 1
    return c


def brute_force_dos(L):
    """g(m) by enumeration of all 2^(L*L) states (L = 4: 65536 states)."""
    N = L * L
    assert N <= 20
    idx = np.arange(1 << N, dtype=np.int64)
    s = (((idx[:, None] >> np.arange(N)) & 1) * 2 - 1).astype(np.int8).reshape(-1, L, L)
    e = -(s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    m = (e + 2 * N) // 4
    return np.bincount(m, minlength=N + 1).astype(np.int64)


@functools.lru_cache(maxsize=None)
def transfer_dos(L):
    """Exact g(m) for an even L x L torus by a row transfer matrix.

    Rows are L-bit words; a row contributes popcount(a ^ rot(a)) horizontal
    broken bonds and a pair of rows popcount(a ^ b) vertical ones.  The trace
    over the first row is taken over cyclic-shift classes (the torus is
    translation invariant along x), with multiplicity.  Intermediate sums stay
    below 2^53 for L <= 8, so the float64 matrix products are exact; the
    closing step is done in int64.
    """
    assert L % 2 == 0 and 2 <= L <= 8
    S = 1 << L
    N = L * L
    maxb = 2 * N
    a = np.arange(S, dtype=np.int64)
    rot = ((a << 1) | (a >> (L - 1))) & (S - 1)
    hrow = _popcount(a ^ rot)
    vb = _popcount(a[:, None] ^ a[None, :])
    masks = [(vb == d).astype(np.float64) for d in range(L + 1)]
    # cyclic-shift class representatives of the first row
    seen = np.zeros(S, dtype=bool)
    reps = []
    for r in range(S):
        if seen[r]:
            continue
        orbit = set()
        x = r
        for _ in range(L):
            orbit.add(x)
            x = ((x << 1) | (x >> (L - 1))) & (S - 1)
        for o in orbit:
            seen[o] = True
        reps.append((r, len(orbit)))
    g = np.zeros(maxb + 1, dtype=np.int64)
    for a0, mult in reps:
        v = np.zeros((S, maxb + 1), dtype=np.float64)
        v[a0, hrow[a0]] = 1.0
        for _ in range(1, L):
            new = np.zeros_like(v)
            for d in range(L + 1):
                c = masks[d] @ v  # c[b, e] = sum over a with popcount(a^b) = d of v[a, e]
                for hb in np.unique(hrow):
                    sel = hrow == hb
                    sh = d + int(hb)
                    if sh <= maxb:
                        new[sel, sh:] += c[sel, : maxb + 1 - sh]
            v = new
        vi = np.rint(v).astype(np.int64)
        for last in range(S):
            sh = int(vb[last, a0])
            g[sh:] += mult * vi[last, : maxb + 1 - sh]
    # broken bonds -> level
    assert np.all(g[1::2] == 0)
    return g[0::2].copy()


def kaufman_lnZ(L, K, prec=300):
    """ln Z of the L x L periodic Ising model at coupling K = beta J (Kaufman)."""
    with mpmath.workprec(prec):
        K = mpmath.mpf(K)
        m = n = L
        c = mpmath.cosh(2 * K) * mpmath.coth(2 * K)

        def gam(l):
            if l == 0:
                return 2 * K + mpmath.log(mpmath.tanh(K))  # signed
            return mpmath.acosh(c - mpmath.cos(mpmath.pi * l / n))

        z1 = z2 = z3 = z4 = mpmath.mpf(1)
        for r in range(n):
            go, ge = gam(2 * r + 1), gam(2 * r)
            z1 *= 2 * mpmath.cosh(m * go / 2)
            z2 *= 2 * mpmath.sinh(m * go / 2)
            z3 *= 2 * mpmath.cosh(m * ge / 2)
            z4 *= 2 * mpmath.sinh(m * ge / 2)
        Z = mpmath.mpf(0.5) * (2 * mpmath.sinh(2 * K)) ** (m * n / mpmath.mpf(2)) * (z1 + z2 + z3 + z4)
        return mpmath.log(Z)


def lnZ_from_dos(g, L, K, prec=300):
    """ln sum_m g(m) exp(-K E(m)) with E = 4m - 2N."""
    N = L * L
    with mpmath.workprec(prec):
        K = mpmath.mpf(K)
        z = mpmath.fsum(int(gm) * mpmath.exp(-K * (4 * mm - 2 * N)) for mm, gm in enumerate(g) if gm)
        return mpmath.log(z)


def mean_energy_exact(L, K):
    """<E> = -d lnZ / dK from Kaufman's form (central difference at 300 bits)."""
    with mpmath.workprec(300):
        K = mpmath.mpf(K)
        h = mpmath.mpf("1e-40")
        return float(-(kaufman_lnZ(L, K + h) - kaufman_lnZ(L, K - h)) / (2 * h))


def bin_dos(g, bin_shift):
    """Sum a level density of states into bins of 2^bin_shift levels."""
    nb = ((len(g) - 1) >> bin_shift) + 1
    G = np.zeros(nb, dtype=object)
    for m, gm in enumerate(g):
        G[m >> bin_shift] += int(gm)
    return G
