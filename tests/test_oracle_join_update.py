"""Pins of the oracle's joint (Algorithm steps 3-5), weight update (eq.
new_weight) and recursion (Sec. 4.2).

Hand-built traces with weights whose differences are either >= 0 (always
accepted) or <= -100 (threshold 0: accepted only by the word 0, checked absent)
give the joint's cut points exactly; the remaining cases are the closed forms
and invariants of the update, and the recursion's convergence to the exact
density of states.
"""
import math

import mpmath
import numpy as np

from paper_0812_2964_amd import exact as X
import oracle as O

SEED = 1


def _no_zero_words(L, r, p, M):
    for i in range(p):
        for k in range(M):
            assert O.uniform(SEED, L, 2, r, i, k) != 0


def test_join_hand_built_cuts():
    L, bs = 4, 0  # levels 0..16, one bin per level
    N = 16
    lnW = np.zeros(N + 1)
    lnW[10:] = -200.0  # levels >= 10 are "heavy-penalty": moving there from < 10 is never accepted
    M = 6
    # trace values are E/4 = m - N/2
    lv = np.array([
        [3, 4, 12, 5, 6, 7],      # chain 0: kept whole (first seam is none)
        [11, 12, 4, 12, 5, 8],    # vs seam 7: 11, 12 rejected, first accepted at k=3
        [14, 13, 12, 11, 10, 15], # vs seam 8: all rejected -> cut -1, seam stays 8
        [12, 2, 3, 3, 3, 9],      # vs seam 8 (carried): 12 rejected, k=2 accepted
    ])
    tr = lv - N // 2
    _no_zero_words(L, 0, 4, M)
    cut, H, ret, sigma = O.join(L, bs, SEED, tr, lnW, -1, 0)
    assert list(cut) == [1, 3, -1, 2]
    assert sigma == 9
    want = np.zeros(N + 1, dtype=np.int64)
    for row, c in zip(lv, cut):
        if c > 0:
            for v in row[c - 1:]:
                want[v] += 1
    assert np.array_equal(H, want)
    assert ret == 6 + 4 + 0 + 5 == H.sum()
    # naive splice (mode 1) keeps everything
    cut1, H1, ret1, sig1 = O.join(L, bs, SEED, tr, lnW, -1, 0, mode=1)
    assert list(cut1) == [1, 1, 1, 1] and ret1 == 24 and sig1 == 9
    # a carried seam from a previous round applies to chain 0
    _no_zero_words(L, 5, 4, M)
    cut2, _, _, _ = O.join(L, bs, SEED, tr, lnW, 12, 5)
    assert cut2[0] == 1  # seam at level 12 (heavy); moving to 3 is uphill in weight: accepted


def test_join_lnW_zero_keeps_everything():
    R = O.Run(8, 8, seed=SEED, bin_shift=1)
    tr, hist = R.run(50)
    cut, H = R.join(tr)
    assert np.all(cut == 1)
    assert np.array_equal(H, hist)
    assert R.sigma == tr[-1, -1] + 32


def test_join_acceptance_probability_is_metropolis():
    # Each chain is (level 2, level 0) with ln w(2) - ln w(0) = ln 0.3 and the
    # seam at level 0.  The first test accepts with probability
    # (tau + 1) / 2^32 = 0.3; otherwise level 0 is accepted at k = 2.  Either
    # way the next seam is level 0 again, so every chain sees the same test.
    L, bs, N = 4, 0, 16
    lnW = np.zeros(N + 1)
    lnW[2] = math.log(0.3)
    p = 20000
    tr = np.tile(np.array([2 - N // 2, 0 - N // 2]), (p, 1))
    cut, H, ret, sigma = O.join(L, bs, SEED, tr, lnW, 0, 0)
    assert set(np.unique(cut)) == {1, 2} and sigma == 0
    frac = (cut == 1).mean()
    assert abs(frac - 0.3) < 0.015
    assert ret == H.sum() == (cut == 1).sum() * 2 + (cut == 2).sum()


def test_update_closed_forms():
    L, bs = 8, 1
    nb = O.n_bins(L, bs)
    rng = np.random.default_rng(0)
    lnW = rng.normal(0, 5, nb)
    H = np.full(nb, 1000, dtype=np.int64)
    w, flat = O.update(L, bs, H, lnW)
    assert np.all(w == lnW - O.det_log(1000))
    assert flat
    H = np.zeros(nb, dtype=np.int64)
    w, flat = O.update(L, bs, H, lnW)
    assert np.array_equal(w, lnW) and not flat
    H = rng.integers(0, 50, nb)
    H[3] = 0
    w, _ = O.update(L, bs, H, lnW)
    for b in range(nb):
        want = lnW[b] - math.log(H[b]) if H[b] > 0 else lnW[b]
        assert abs(w[b] - want) <= 4e-16 * max(1.0, abs(want))


def test_flatness_integer_rule():
    L, bs = 4, 0  # 17 levels, 15 reachable (m = 1, 15 excluded)
    nb = 17
    reach = O.reachable_bins(L, bs)
    assert reach.sum() == 15 and not reach[1] and not reach[15]
    H = np.zeros(nb, dtype=np.int64)
    H[reach] = 100
    assert O.update(L, bs, H, np.zeros(nb))[1]
    H[0] = 80  # min/mean = 80/98.67 = 0.81 >= 0.8
    assert O.update(L, bs, H, np.zeros(nb))[1]
    H[0] = 79  # 5*15*79 = 5925 >= 4*1479 = 5916: still flat
    assert O.update(L, bs, H, np.zeros(nb))[1]
    H[0] = 78  # 5*15*78 = 5850 < 4*1478 = 5912: not flat
    assert not O.update(L, bs, H, np.zeros(nb))[1]
    H[0] = 100
    H[1] = 0  # unreachable bin is ignored
    assert O.update(L, bs, H, np.zeros(nb))[1]


def test_recursion_converges_to_exact_dos_L8():
    # The recursion of Sec. 3.1 run as in Sec. 4.2 (L = 8, 16 chains,
    # 10^4 sweeps per iteration, width-8 energy bins): ln w + ln G is flat.
    R = O.Run(8, 16, seed=SEED, bin_shift=1)
    G = X.bin_dos(X.transfer_dos(8), 1)
    lnG = np.array([float(mpmath.log(int(v))) for v in G])
    flat_at = None
    for it in range(10):
        tr, _ = R.run(10000)
        R.join(tr)
        if R.update() and flat_at is None:
            flat_at = it + 1
    d = R.lnW + lnG
    assert flat_at is not None and flat_at <= 10
    assert d.max() - d.min() < 0.35


def test_recursion_converges_to_exact_dos_L4_levels():
    R = O.Run(4, 8, seed=3, bin_shift=0)
    g = X.brute_force_dos(4)
    for it in range(25):
        tr, _ = R.run(4000)
        R.join(tr)
        R.update()
    reach = g > 0
    d = (R.lnW + np.log(np.maximum(g, 1)))[reach]
    assert d.max() - d.min() < 0.15


def test_blockwise_joint_equals_the_whole():
    """A run split into two blocks of chains (chain offsets 0 and p/2) makes
    the same traces as the whole run, and joining the blocks in turn, the
    second from the seam the first ended with, keeps exactly what one joint
    over all chains keeps -- the exchange a run split over several GPUs
    needs.  Three rounds, a non-trivial weight, detailed balance and the
    naive splice."""
    L, p, M, bs = 8, 12, 25, 1
    # a weight and round count for which starting a block from any other seam
    # (its own end of the round before, say) changes the cut points
    rng = np.random.default_rng(13)
    lnW = rng.normal(0, 3.0, O.n_bins(L, bs))
    for mode in (0, 1):
        whole = O.Run(L, p, seed=4, bin_shift=bs, lnW=lnW)
        parts = [O.Run(L, p // 2, seed=4, bin_shift=bs, lnW=lnW, chain_offset=o) for o in (0, p // 2)]
        for _ in range(3):
            tr, _ = whole.run(M)
            cut, H = whole.join(tr, mode)
            trs = [q.run(M)[0] for q in parts]
            assert np.array_equal(np.concatenate(trs), tr)
            parts[0].sigma = parts[1].sigma  # each round starts where the last block ended (step 4)
            c0, H0 = parts[0].join(trs[0], mode)
            parts[1].sigma = parts[0].sigma
            c1, H1 = parts[1].join(trs[1], mode)
            assert np.array_equal(np.concatenate([c0, c1]), cut)
            assert np.array_equal(H0 + H1, H)
            assert parts[1].sigma == whole.sigma
        assert parts[0].retained + parts[1].retained == whole.retained
