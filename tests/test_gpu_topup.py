"""GPU parity of the energy-ordered joint (mc_join mode 2) and of Algorithm
step 6's top-up iteration (mc_iterate_topup) against the oracle, bit for bit;
the int64 histogram of an iteration beyond 2^31 configurations; argument
errors."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402

pytestmark = pytest.mark.gpu


def _mc():
    import paper_0812_2964_amd as mc

    return mc


def _weight(L, bs, seed, amp=3.0):
    rng = np.random.default_rng(seed)
    nb = ((L * L) >> bs) + 1
    x = (np.arange(nb) - nb / 2) / nb
    return -0.5 * L * L * x * x + rng.normal(0, amp, nb)


@pytest.mark.parametrize("L,P,M,bs", [(8, 16, 30, 1), (16, 100, 20, 0), (32, 1500, 8, 1), (100, 700, 2, 1),
                                      (256, 33, 1, 0)])
def test_energy_ordered_joint_bitexact(L, P, M, bs):
    """Several rounds of sweeps and mode-2 joints (the order built on the
    device); 1500 chains cross the serial fix-up's chunk of 1024 positions
    and the ordering's chunks of 256; L = 256 has int32 traces and 65537
    levels (the ordering's bitmaps at their largest)."""
    import torch

    mc = _mc()
    w = _weight(L, bs, L)
    ctx = mc.Context([(L, P, 5, bs)])
    ctx.init_weights(w)
    R = O.Run(L, P, seed=5, bin_shift=bs, lnW=w)
    h = ctx.new_hist()
    for rnd in range(3):
        tr, cut = ctx.new_trace(M), ctx.new_cut()
        ctx.run_chains(M, tr, h)
        ctx.join(tr, cut, h, mode=2)
        otr, _ = R.run(M)
        ocut, oH = R.join(otr, mode=2)
        assert np.array_equal(tr.cpu().numpy().astype(np.int32), otr), "trace, round %d" % rnd
        assert np.array_equal(cut.cpu().numpy(), ocut), "cut, round %d" % rnd
        torch.cuda.synchronize()
    assert np.array_equal(h.cpu().numpy(), R.H), "joined histogram"
    w2, flat, ret = ctx.update_weights(h)
    oret = R.retained
    oflat = R.update()
    assert ret == oret and flat == oflat
    assert np.array_equal(w2.view(np.uint64), R.lnW.view(np.uint64))
    ctx.close()


def test_energy_ordered_graph_replays_equal_eager_iterations():
    """Iterations with energy-ordered joints captured in a graph (the order
    is built on the device, so the whole iteration is captured) equal the
    same iterations made eagerly, bit for bit, with eager work between the
    replays."""
    import torch

    mc = _mc()
    L, P, M, bs = 16, 200, 40, 1
    w = _weight(L, bs, 3)
    a = mc.Context([(L, P, 5, bs)])
    b = mc.Context([(L, P, 5, bs)])
    a.init_weights(w)
    b.init_weights(w)
    tr, h, cut = a.new_trace(M), a.new_hist(), a.new_cut()
    g = a.graph(M, 2, [tr], [h], [cut], mode=2)
    for rep in range(3):
        g.launch()
        a.sync()
        scratch = torch.ones(1 << 20, device="cuda").sum()  # eager work between replays
        for it in range(2):
            tb, hb, cb = b.new_trace(M), b.new_hist(), b.new_cut()
            b.run_chains(M, tb, hb)
            b.join(tb, cb, hb, mode=2)
            b.update_weights(hb, want=False)
        assert float(scratch) == float(1 << 20)
        assert np.array_equal(tr.cpu().numpy(), tb.cpu().numpy()), rep
        assert np.array_equal(cut.cpu().numpy(), cb.cpu().numpy()), rep
        assert np.array_equal(a.weights().view(np.uint64), b.weights().view(np.uint64)), rep
        assert a.counters() == b.counters() and np.array_equal(a.levels(), b.levels())
    g.close()
    a.close()
    b.close()


@pytest.mark.parametrize("mode", [0, 2])
def test_topup_iteration_bitexact(mode):
    """Three iterations with top-up rounds (the totals need several rounds of
    different lengths) against the oracle's iterate_topup."""
    import torch

    mc = _mc()
    L, P, bs, m_max = 16, 64, 1, 60
    w = _weight(L, bs, 7, amp=4.0)
    ctx = mc.Context([(L, P, 9, bs)])
    ctx.init_weights(w)
    R = O.Run(L, P, seed=9, bin_shift=bs, lnW=w)
    tr, h, cut = ctx.new_trace(m_max), ctx.new_hist(), ctx.new_cut()
    for it, m_total in enumerate((P * 150, P * 45, P * 200)):
        rounds, sweeps, kept, flat = ctx.iterate_topup(m_total, m_max, tr, h, cut, mode=mode)
        orounds, oret, oflat, otraces = R.iterate_topup(m_total, m_max, mode=mode)
        assert rounds == len(orounds) and sweeps == sum(orounds), (it, rounds, orounds)
        assert kept == oret and kept >= m_total and flat == oflat
        last = otraces[-1]
        got = tr.view(-1)[: P * last.shape[1]].view(P, last.shape[1]).cpu().numpy().astype(np.int32)
        assert np.array_equal(got, last), "last round's trace, iteration %d" % it
        assert np.array_equal(ctx.weights().view(np.uint64), R.lnW.view(np.uint64)), "ln w, iteration %d" % it
        assert not h.cpu().numpy().any()
        torch.cuda.synchronize()
    ctx.close()


def test_topup_histogram_beyond_int32():
    """4096 chains at L = 4 from ln w = 0: every joint accepts, so the
    iteration keeps all 4096 x 1.1e6 = 4.5e9 configurations (rounds of 5e5,
    5e5 and 1e5 sweeps); the update's ln w then counts them all,
    sum_b exp(-ln w_b) = 4.5e9, which an int32 histogram could not hold."""
    import torch

    mc = _mc()
    L, P, m_max = 4, 4096, 500000
    m_total = P * 1100000
    ctx = mc.Context([(L, P, 1, 0)])
    tr = torch.empty((P, m_max), dtype=torch.int16, device="cuda")
    h, cut = ctx.new_hist(), ctx.new_cut()
    rounds, sweeps, kept, flat = ctx.iterate_topup(m_total, m_max, tr, h, cut, mode=0)
    assert (rounds, sweeps, kept) == (3, 1100000, m_total)
    w = ctx.weights()
    assert np.isfinite(w).all()
    total = np.exp(-w[w != 0]).sum()
    assert total == pytest.approx(m_total, rel=1e-9)
    assert total > 2**31
    ctx.close()


def test_topup_argument_errors():
    import torch

    mc = _mc()
    ctx = mc.Context([(8, 4, 1, 1), (16, 4, 1, 1)])
    tr = torch.zeros((4, 10), dtype=torch.int16, device="cuda")
    with pytest.raises(mc.MCError):
        ctx.iterate_topup(40, 10, tr, ctx.new_hist(), ctx.new_cut())  # two sizes
    ctx.close()
    ctx = mc.Context([(8, 4096, 1, 1)])
    big = 600000
    with pytest.raises(mc.MCError):  # 4096 x 600000 > 2^31 - 1
        _raw_topup(ctx, 10, big)
    tr = torch.zeros((4096, 10), dtype=torch.int16, device="cuda")
    h, cut = ctx.new_hist(), ctx.new_cut()
    for bad in (dict(m_total=0, m_max=10), dict(m_total=10, m_max=10, mode=3), dict(m_total=10, m_max=10,
                                                                                      max_rounds=0)):
        with pytest.raises(mc.MCError):
            ctx.iterate_topup(bad["m_total"], bad["m_max"], tr, h, cut, mode=bad.get("mode", 0),
                              max_rounds=bad.get("max_rounds", 1000))
    # a run since the last update: the iteration must start after an update
    ctx.run_chains(10, tr, h)
    with pytest.raises(mc.MCError):
        ctx.iterate_topup(10, 10, tr, h, cut)
    ctx.close()


def _raw_topup(ctx, m_total, m_max):
    """Call the entry point with a trace too small for m_max: it must fail on
    the histogram bound before touching any buffer."""
    import ctypes

    import torch

    mc = _mc()
    tr = torch.zeros(16, dtype=torch.int16, device="cuda")
    h, cut = ctx.new_hist(), ctx.new_cut()
    st = mc.lib().mc_iterate_topup(ctx._h, m_total, m_max, 10, ctypes.c_void_p(tr.data_ptr()),
                                   ctypes.c_void_p(h.data_ptr()), ctypes.c_void_p(cut.data_ptr()), 0, None, None, None,
                                   None)
    mc._check(st)
