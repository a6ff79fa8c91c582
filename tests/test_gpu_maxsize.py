"""The largest chain count a size takes (2^20 chains) in the default launch
configuration: 65536 blocks of the quad kernel at L = 32 and the streamed-row
kernel at L = 128.  Sampled chains are replayed by the oracle bit for bit
(trace, final spins and level); the joint of Sec. 2 over all 2^20 chains, its
histogram and the weight update of Eq. (new_weight) are recomputed by the
oracle from the device's traces and must agree exactly."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402

pytestmark = pytest.mark.gpu

P = 1 << 20


def _weight(L, bs, seed, amp):
    rng = np.random.default_rng(seed)
    nb = ((L * L) >> bs) + 1
    x = (np.arange(nb) - nb / 2) / nb
    return -0.5 * L * L * x * x + rng.normal(0, amp, nb)


@pytest.mark.parametrize("L,M,kind", [(32, 200, 7), (128, 8, 8)])
def test_max_chains_rounds(L, M, kind):
    import paper_0812_2964_amd as mc
    import torch

    print("max chains: L=%d P=%d M=%d" % (L, P, M), flush=True)
    bs = 1
    w = _weight(L, bs, L, 2.0)
    ctx = mc.Context([(L, P, 3, bs)])
    assert ctx.launch()[1] == kind
    ctx.init_weights(w)
    N = L * L
    sample = [0, 1, 15, 16, 63, 64, P // 2, P - 2, P - 1]
    sample += np.random.default_rng(L).integers(0, P, 4).tolist()
    state = {}
    for c in sample:
        s0 = O.init_chain(L, 3, c)
        state[c] = (s0, (O.energy(L, s0) + 2 * N) // 4)
    h = ctx.new_hist()
    sigma, lnW = -1, w.copy()
    for rnd in range(2):
        tr, cut = ctx.new_trace(M), ctx.new_cut()
        ctx.run_chains(M, tr, h)
        raw = h.cpu().numpy().copy()
        ctx.join(tr, cut, h)
        torch.cuda.synchronize()
        trace = tr.cpu().numpy().astype(np.int32)
        gcut = cut.cpu().numpy()
        joined = h.cpu().numpy()
        del tr
        # every configuration of the round is in the raw histogram
        assert raw.sum() == P * M
        for c in sample:
            s, m, otr, _ = O.sweeps(L, 3, bs, c, state[c][0], state[c][1], rnd * M, M, lnW)
            assert np.array_equal(trace[c], otr), (rnd, c)
            state[c] = (s, m)
        ocut, oH, oret, sigma = O.join(L, bs, 3, trace, lnW, sigma, rnd, mode=0)
        del trace
        assert np.array_equal(gcut, ocut), rnd
        assert np.array_equal(joined, oH), rnd
        w2, flat, ret = ctx.update_weights(h)
        assert ret == oret
        lnW, oflat = O.update(L, bs, oH, lnW)
        assert flat == oflat
        assert np.array_equal(w2.view(np.uint64), lnW.view(np.uint64)), rnd
        h = ctx.new_hist()
    levels = ctx.levels()
    for c in sample:
        assert np.array_equal(ctx.spins(c), state[c][0]) and levels[c] == state[c][1], c
    ctx.close()
