"""Rounds made in several launches (mc_run_chains_part), the 2^32 limits of
the random words' counters, the recursion statistics (mc_get_stats) and the
level check (mc_check_levels), through the C ABI.

A round of M sweeps made in parts must be bit for bit the round made in one
launch (same random words: the sweep index is the global counter of Algorithm
step 2's chains), and the oracle confirms the sweeps at the very top of the
sweep counter's range."""
import ctypes
import struct
import zlib

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def _mc():
    import paper_0812_2964_amd as mc

    return mc


def _np(t):
    return t.detach().cpu().numpy()


def _weight(L, bs, seed, amp):
    rng = np.random.default_rng(seed)
    nb = ((L * L) >> bs) + 1
    x = (np.arange(nb) - nb / 2) / nb
    return -0.4 * L * L * x * x + rng.normal(0, amp, nb)


@pytest.mark.parametrize("sizes,parts", [
    ([(32, 70, 1, 1)], [3, 10, 1, 6]),
    ([(128, 40, 2, 1)], [2, 1, 3]),
    ([(16, 33, 1, 1), (48, 20, 1, 0)], [5, 4, 1]),
])
def test_round_in_parts_equals_one_launch(sizes, parts):
    mc = _mc()
    M = sum(parts)
    a = mc.Context(sizes)
    b = mc.Context(sizes)
    for i, s in enumerate(sizes):
        w = _weight(s[0], s[3], 7 + i, 1.0)
        a.init_weights(w, i)
        b.init_weights(w, i)
    for rnd in range(2):
        ta = [a.new_trace(M, i) for i in range(len(sizes))]
        ha = [a.new_hist(i) for i in range(len(sizes))]
        tb = [b.new_trace(M, i) for i in range(len(sizes))]
        hb = [b.new_hist(i) for i in range(len(sizes))]
        a.run_chains(M, ta, ha)
        col = 0
        for k, n in enumerate(parts):
            if k + 1 < len(parts):
                # a round in progress cannot be joined or checkpointed
                b.run_chains_part(n, col, tb, hb)
                col += n
                with pytest.raises(mc.MCError) as e:
                    b.join(tb[0], b.new_cut(0), hb[0])
                assert e.value.status == mc.MC_ESTATE
                with pytest.raises(mc.MCError) as e:
                    b.get_state()
                assert e.value.status == mc.MC_ESTATE
            else:
                # a part that does not continue the round is refused
                with pytest.raises(mc.MCError) as e:
                    b.run_chains_part(1, col - 1, tb, hb)
                assert e.value.status == mc.MC_ESTATE
                b.run_chains_part(n, col, tb, hb)
        for i in range(len(sizes)):
            assert np.array_equal(_np(ta[i]), _np(tb[i])), (rnd, i)
            assert np.array_equal(_np(ha[i]), _np(hb[i])), (rnd, i)
            ca, cb = a.new_cut(i), b.new_cut(i)
            a.join(ta[i], ca, ha[i], 0, i)
            b.join(tb[i], cb, hb[i], 0, i)
            assert np.array_equal(_np(ca), _np(cb))
            wa, fa, ra = a.update_weights(ha[i], i)
            wb, fb, rb = b.update_weights(hb[i], i)
            assert np.array_equal(wa.view(np.uint64), wb.view(np.uint64)) and fa == fb and ra == rb
            assert np.array_equal(a.levels(i), b.levels(i))
            assert a.counters(i) == b.counters(i)
    a.close()
    b.close()


def _set_counters(blob, g=None, r=None):
    """A state blob of a one-size context with its sweep / round counters
    replaced, the CRC-32 (zlib) recomputed."""
    b = bytearray(blob)
    at = 24
    if g is not None:
        b[at + 44: at + 48] = struct.pack("<I", g)
    if r is not None:
        b[at + 48: at + 52] = struct.pack("<I", r)
    b[8:12] = b"\0\0\0\0"
    b[8:12] = struct.pack("<I", zlib.crc32(bytes(b)) & 0xFFFFFFFF)
    return bytes(b)


def test_sweep_counter_limit_and_the_top_of_its_range():
    """The last 10 sweep indices below 2^32 are usable and give the oracle's
    sweeps; one more is refused (the random words would repeat)."""
    mc = _mc()
    L, P, N = 16, 9, 256
    w = _weight(L, 1, 3, 1.0)
    ctx = mc.Context([(L, P, 1, 1)])
    ctx.init_weights(w)
    g0 = (1 << 32) - 10
    ctx.set_state(_set_counters(ctx.get_state(), g=g0))
    assert ctx.counters()[2] == g0
    tr, h = ctx.new_trace(11), ctx.new_hist()
    tp = (ctypes.c_void_p * 1)(tr.data_ptr())
    hp = (ctypes.c_void_p * 1)(h.data_ptr())
    assert mc.lib().mc_run_chains(ctx._h, 11, tp, hp) == mc.MC_EOVERFLOW
    M = 10
    tr = ctx.new_trace(M)
    ctx.run_chains(M, tr, h)
    got = _np(tr).astype(np.int32)
    for c in range(P):
        s0 = O.init_chain(L, 1, c)
        m0 = (O.energy(L, s0) + 2 * N) // 4
        _, _, otr, _ = O.sweeps(L, 1, 1, c, s0, m0, g0, M, w)
        assert np.array_equal(got[c], otr), c
    cut = ctx.new_cut()
    ctx.join(tr, cut, h)
    ctx.update_weights(h, want=False)
    # every sweep index is used: nothing more may run
    with pytest.raises(mc.MCError) as e:
        ctx.run_chains(1, ctx.new_trace(1), h)
    assert e.value.status == mc.MC_EOVERFLOW
    # a graph cannot be replayed past the limit either
    ctx2 = mc.Context([(L, P, 1, 1)])
    ctx2.set_state(_set_counters(ctx2.get_state(), g=(1 << 32) - 100))
    trs, hs, cuts = [ctx2.new_trace(60)], [ctx2.new_hist()], [ctx2.new_cut()]
    g = ctx2.graph(60, 1, trs, hs, cuts)
    g.launch()
    ctx2.sync()
    with pytest.raises(mc.MCError) as e:
        g.launch()
    assert e.value.status == mc.MC_EOVERFLOW
    g.close()
    ctx2.close()
    ctx.close()


def test_round_counter_limit():
    mc = _mc()
    ctx = mc.Context([(8, 4, 1, 1)])
    ctx.set_state(_set_counters(ctx.get_state(), r=(1 << 32) - 1))
    tr, h, cut = ctx.new_trace(5), ctx.new_hist(), ctx.new_cut()
    ctx.run_chains(5, tr, h)
    ctx.join(tr, cut, h)  # round 2^32 - 1, the last one
    ctx.run_chains(5, tr, h)
    with pytest.raises(mc.MCError) as e:
        ctx.join(tr, cut, h)
    assert e.value.status == mc.MC_EOVERFLOW
    ctx.close()


@pytest.mark.parametrize("L,P,bs,M", [(8, 16, 1, 300), (32, 40, 1, 200), (100, 6, 1, 3), (256, 2, 1, 1)])
def test_stats_and_level_check_match_the_oracle(L, P, bs, M):
    """mc_get_stats after each iteration against the oracle's histogram, cuts
    and ln w; every chain's level equals half its broken bonds."""
    mc = _mc()
    w = _weight(L, bs, 11, 0.5)
    ctx = mc.Context([(L, P, 1, bs)])
    ctx.init_weights(w)
    R = O.Run(L, P, seed=1, bin_shift=bs, lnW=w)
    reach = O.reachable_bins(L, bs)
    for it in range(3):
        tr, h, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
        ctx.run_chains(M, tr, h)
        ctx.join(tr, cut, h)
        ctx.update_weights(h, want=False)
        otr, _ = R.run(M)
        ocut, _ = R.join(otr)
        H = R.H.copy()
        oret = R.retained
        oflat = R.update()
        st = ctx.stats()
        assert st["updates"] == it + 1
        assert st["last_flat"] == int(oflat)
        assert st["retained_last"] == oret
        assert st["n_reach_bins"] == int(reach.sum())
        assert st["hist_sum"] == int(H[reach].sum()) and st["hist_min"] == int(H[reach].min())
        assert st["lnw_min"] == R.lnW[reach].min() and st["lnw_max"] == R.lnW[reach].max()
        assert st["join_none"] == int((ocut < 0).sum())
        kept = ocut[ocut > 0]
        assert st["join_cut_max"] == int(kept.max(initial=0)) and st["join_cut_sum"] == int(kept.sum())
        assert (st["seam"], st["round_index"], st["sweep_index"]) == (R.sigma, R.r, R.g)
        assert ctx.check_levels() == 0
    ctx.close()
