"""Pins of the oracle's Algorithm step 6 (top-up rounds to M_total) and of the
energy ordering of the chains at the joints (Sec. 2, remarks after the
algorithm).  The paper fixes neither the rule for the next round's length nor
the ordering; the readings are the oracle's (topup_sweeps, energy_order), and
these tests pin them to what must hold for any such reading:

* the ordering is a permutation; it is the index order when the traces are
  already chained by energy, and then the joint equals the plain one;
* with a flat weight every test accepts, so any order keeps every
  configuration and gives the same histogram;
* each position takes a chain whose first level is nearest to the level the
  previous chain ended on (local optimality of the greedy choice);
* the next round's length is the smallest that covers the shortfall at a
  constant, exactly known retention rate;
* the top-up loop stops at the first round that reaches M_total, and with
  M_total within the first round it is the plain iteration.
"""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402


def test_order_is_permutation_and_locally_nearest():
    rng = np.random.default_rng(5)
    for p in (1, 2, 7, 40):
        first = rng.integers(0, 50, p)
        last = rng.integers(0, 50, p)
        for sigma in (-1, 0, 25, 49):
            order = O.energy_order(first, last, sigma)
            assert sorted(order.tolist()) == list(range(p))
            ref = sigma
            start = 0
            if sigma < 0:
                assert order[0] == 0
                ref = last[0]
                start = 1
            for t in range(start, p):
                rest = order[t:]
                d = np.abs(first[rest] - ref)
                c = order[t]
                assert abs(first[c] - ref) == d.min()
                ties = rest[d == d.min()]
                assert first[c] == first[ties].min()
                assert c == ties[first[ties] == first[c]].min()
                ref = last[c]


def test_order_of_energy_chained_traces_is_index_order():
    # chain c starts at level 10 + 3c and ends at 11 + 3c: from the seam 10,
    # each chain's first level is the nearest to where the previous one ended
    L, p, M = 8, 6, 5
    N = L * L
    first = 10 + 3 * np.arange(p)
    tr = np.zeros((p, M), dtype=np.int32)
    for c in range(p):
        tr[c] = np.linspace(first[c], first[c] + 1, M).round().astype(np.int32) - N // 2
    order = O.energy_order(tr[:, 0] + N // 2, tr[:, -1] + N // 2, 10)
    assert order.tolist() == list(range(p))
    rng = np.random.default_rng(2)
    lnW = rng.normal(0, 1.0, N // 2 + 1)
    a = O.join(L, 1, 3, tr, lnW, 10, 4, mode=0)
    b = O.join(L, 1, 3, tr, lnW, 10, 4, mode=2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2:] == b[2:]


def test_flat_weight_keeps_everything_in_any_order():
    L, p, M = 8, 12, 30
    R = O.Run(L, p, seed=7, bin_shift=1)
    tr, raw = R.run(M)
    lnW = np.zeros(O.n_bins(L, 1))
    for sigma in (-1, 5, 40):
        for mode in (0, 2):
            cut, H, ret, _ = O.join(L, 1, 7, tr, lnW, sigma, 0, mode=mode)
            assert (cut == 1).all() and ret == p * M
            assert np.array_equal(H, raw)


def test_histogram_counts_exactly_the_kept_configurations():
    L, p, M = 8, 16, 40
    rng = np.random.default_rng(11)
    lnW = rng.normal(0, 3.0, O.n_bins(L, 1))
    R = O.Run(L, p, seed=2, bin_shift=1, lnW=lnW)
    tr, _ = R.run(M)
    for mode in (0, 2):
        cut, H, ret, _ = O.join(L, 1, 2, tr, lnW, 20, 1, mode=mode)
        assert H.sum() == ret == sum(M - k + 1 for k in cut if k > 0)
        # the histogram is that of the kept suffixes
        ref = np.zeros_like(H)
        for c in range(p):
            if cut[c] > 0:
                for v in tr[c, cut[c] - 1:]:
                    ref[(v + L * L // 2) >> 1] += 1
        assert np.array_equal(H, ref)


@pytest.mark.parametrize("rate", [1, 3, 16])
def test_next_round_covers_the_shortfall_at_a_known_rate(rate):
    m_max = 1000
    for swept in (1, 10, 37):
        kept = rate * swept
        for m_total in (kept + 1, kept + rate, kept + 5 * rate + 1, kept + 10**6):
            m = O.topup_sweeps(m_total, m_max, kept, swept)
            need = m_total - kept
            exact = -(-need // rate)
            assert m == min(m_max, exact)
            if m < m_max:
                assert kept + rate * m >= m_total > kept + rate * (m - 1)
    assert O.topup_sweeps(100, 50, 0, 10) == 50


def test_topup_stops_at_the_first_sufficient_round_and_reduces_to_one_round():
    L, p = 8, 16
    rng = np.random.default_rng(4)
    lnW = rng.normal(0, 4.0, O.n_bins(L, 1))
    for mode in (0, 2):
        A = O.Run(L, p, seed=3, bin_shift=1, lnW=lnW)
        A.run(50)  # a first round so that the joints have a seam
        A.retained = 0
        A.H[:] = 0
        rounds, ret, flat, traces = A.iterate_topup(p * 120, 40, mode=mode)
        assert ret >= p * 120
        assert len(rounds) >= 3 and rounds[0] == 40
        # the rounds before the last did not reach the total
        B = O.Run(L, p, seed=3, bin_shift=1, lnW=lnW)
        B.run(50)
        B.retained = 0
        B.H[:] = 0
        for m in rounds[:-1]:
            tr, _ = B.run(m)
            B.join(tr, mode)
        assert B.retained < p * 120
        # a total within the first round is the plain iteration
        C = O.Run(L, p, seed=3, bin_shift=1, lnW=lnW)
        D = O.Run(L, p, seed=3, bin_shift=1, lnW=lnW)
        for X in (C, D):
            X.run(50)
            X.retained = 0
            X.H[:] = 0
        rounds, ret, flat, _ = C.iterate_topup(1, 30, mode=mode)
        tr, _ = D.run(30)
        D.join(tr, mode)
        d_ret = D.retained
        d_flat = D.update()
        assert rounds == [30] and ret == d_ret and flat == d_flat
        assert np.array_equal(C.lnW.view(np.uint64), D.lnW.view(np.uint64))
