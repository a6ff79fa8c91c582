"""GPU path (through the C ABI) against the CPU oracle, element by element.

Integer outputs (energy traces, histograms, cut points, seams, lattices,
levels) must be identical; ln w after an update must be identical bit for bit
(both sides evaluate ln with the same fixed sequence of binary64 operations).
"""
import os

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _mc():
    import paper_0812_2964_amd as mc

    return mc


def _np(t):
    return t.detach().cpu().numpy()


def gpu_round(ctx, M, i=0, mode=0, update=True, hist=None):
    """One round of a one-size context: run, join, and (optionally) update.
    hist carries the joint histogram across rounds that are not followed by
    an update (Algorithm step 6)."""
    tr = ctx.new_trace(M, i)
    h = hist if hist is not None else ctx.new_hist(i)
    cut = ctx.new_cut(i)
    ctx.run_chains(M, tr, h)
    raw = _np(h).copy()
    ctx.join(tr, cut, h, mode, i)
    joined = _np(h).copy()
    out = dict(trace=_np(tr).astype(np.int32), raw=raw, cut=_np(cut), joined=joined)
    if update:
        w, flat, ret = ctx.update_weights(h, i)
        out.update(lnW=w, flat=flat, retained=ret, hist_after=_np(h).copy())
    return out


def oracle_round(R, M, mode=0, update=True):
    H0 = R.H.copy()
    tr, raw = R.run(M)
    cut, H = R.join(tr, mode)
    out = dict(trace=tr, raw=raw + H0, cut=cut, joined=R.H.copy(), retained=R.retained)
    if update:
        out["flat"] = R.update()
        out["lnW"] = R.lnW.copy()
    return out


def assert_round_equal(g, o, update=True):
    assert np.array_equal(g["trace"], o["trace"]), "trace differs"
    assert np.array_equal(g["raw"], o["raw"]), "raw histogram differs"
    assert np.array_equal(g["cut"], o["cut"]), "cut points differ"
    assert np.array_equal(g["joined"], o["joined"]), "joined histogram differs"
    if update:
        assert g["retained"] == o["retained"]
        assert g["flat"] == o["flat"]
        assert np.array_equal(g["lnW"].view(np.uint64), o["lnW"].view(np.uint64)), "ln w differs"
        assert not g["hist_after"].any()


def assert_state_equal(ctx, R, i=0):
    assert np.array_equal(ctx.levels(i), R.m)
    for c in sorted({0, R.p // 2, R.p - 1}):
        assert np.array_equal(ctx.spins(c, i), R.spins[c])
    seam, rnd, sweep = ctx.counters(i)
    assert (seam, rnd, sweep) == (R.sigma, R.r, R.g)


def test_initial_state_matches_oracle():
    mc = _mc()
    for L, P in [(8, 16), (32, 70), (6, 5), (128, 3)]:
        ctx = mc.Context([(L, P, 1, 1)])
        R = O.Run(L, P, seed=1, bin_shift=1)
        assert np.array_equal(ctx.levels(), R.m)
        for c in range(P):
            assert np.array_equal(ctx.spins(c), R.spins[c])
        ctx.close()


def test_config_L8_16chains_full_recursion_bitexact():
    """L = 8, 16 chains, 10^4 sweeps per iteration, 10 iterations of the
    recursion from ln w = 0, width-8 bins (33 bins), seed 1."""
    mc = _mc()
    ctx = mc.Context([(8, 16, 1, 1)])
    R = O.Run(8, 16, seed=1, bin_shift=1)
    ctx.init_weights(None)
    flats = []
    for it in range(10):
        g = gpu_round(ctx, 10000)
        o = oracle_round(R, 10000)
        assert_round_equal(g, o)
        flats.append(g["flat"])
    assert_state_equal(ctx, R)
    assert any(flats)  # this workload reaches a flat histogram within 10 iterations
    ctx.close()


def _prior_lnW():
    return np.load(os.path.join(HERE, "golden", "lnW_L32_prior.npy"))


def test_L32_prior_weight_rounds_bitexact():
    mc = _mc()
    P = 130  # two full blocks of 64 and a ragged tail
    ctx = mc.Context([(32, P, 1, 1)])
    w = _prior_lnW()
    ctx.init_weights(w)
    R = O.Run(32, P, seed=1, bin_shift=1, lnW=w)
    h = ctx.new_hist()
    for M, upd in [(150, False), (97, True), (64, True)]:
        g = gpu_round(ctx, M, update=upd, hist=h)
        o = oracle_round(R, M, update=upd)
        assert_round_equal(g, o, update=upd)
    assert_state_equal(ctx, R)
    ctx.close()


@pytest.mark.parametrize("L,P,bs,M", [(4, 65, 0, 40), (6, 9, 1, 30), (10, 9, 0, 20), (12, 64, 1, 30),
                                      (16, 70, 1, 25), (24, 33, 1, 12), (48, 20, 1, 6), (64, 40, 1, 5),
                                      (64, 7, 0, 4), (128, 5, 1, 2), (128, 9, 0, 2), (256, 20, 1, 1)])
def test_sizes_and_binnings_bitexact(L, P, bs, M):
    mc = _mc()
    N = L * L
    nb = (N >> bs) + 1
    rng = np.random.default_rng(L * 7 + bs)
    # a smooth, non-trivial weight: favours the middle of the energy range and
    # rejects a good share of moves
    x = (np.arange(nb) - nb / 2) / nb
    w = -0.25 * N * x * x + rng.normal(0, 0.3, nb)
    ctx = mc.Context([(L, P, 5, bs)])
    ctx.init_weights(w)
    R = O.Run(L, P, seed=5, bin_shift=bs, lnW=w)
    for _ in range(2):
        g = gpu_round(ctx, M)
        o = oracle_round(R, M)
        assert_round_equal(g, o)
    assert_state_equal(ctx, R)
    ctx.close()


def _smooth_weight(L, bs, seed):
    N = L * L
    nb = (N >> bs) + 1
    rng = np.random.default_rng(seed)
    x = (np.arange(nb) - nb / 2) / nb
    return -0.25 * N * x * x + rng.normal(0, 0.3, nb)


@pytest.mark.parametrize("L,bs,cpb,kind", [(128, 1, None, 8), (128, 1, 13, 8), (128, 1, 32, 8), (128, 1, 20, 8),
                                             (128, 1, 40, 5), (128, 1, 64, 6), (128, 0, 16, 9), (256, 1, None, 9),
                                             (256, 1, 5, 9), (256, 1, 32, 9), (100, 1, None, 8), (100, 1, 32, 8),
                                             (100, 0, 16, 9)])
def test_large_lattice_kernels_bitexact(L, bs, cpb, kind):
    """The streamed-row kernels of the large lattices against the oracle over
    two rounds with a ragged last workgroup: four lanes per chain (the
    default; at most 32 chains per workgroup, 17 or more on two consumer
    waves) with the per-bin thresholds in LDS (kind 8) or, where they do not
    fit (one level per bin at L = 128, L = 256), in global memory (kind 9);
    one lane per chain (more than 32 chains per workgroup) with the table in
    LDS (kind 5) or, where 64 chains leave no room for it, in global memory
    (kind 6).  L = 100 (the paper's lattice) has a partial last word per
    row and runs the four-lane kinds only."""
    mc = _mc()
    P, M = 70, 2
    w = _smooth_weight(L, bs, 11)
    ctx = mc.Context([(L, P, 3, bs)])
    ctx.init_weights(w)
    if cpb is not None:
        ctx.set_chains_per_block(cpb)
    assert ctx.launch()[1] == kind, (cpb, ctx.launch())
    R = O.Run(L, P, seed=3, bin_shift=bs, lnW=w)
    for _ in range(2):
        g = gpu_round(ctx, M)
        o = oracle_round(R, M)
        assert_round_equal(g, o)
    assert_state_equal(ctx, R)
    ctx.close()


def test_join_hand_built_traces_and_modes():
    import torch

    mc = _mc()
    L, N, bs = 4, 16, 0
    lnW = np.zeros(N + 1)
    lnW[10:] = -200.0
    lv = np.array([[3, 4, 12, 5, 6, 7], [11, 12, 4, 12, 5, 8], [14, 13, 12, 11, 10, 15], [12, 2, 3, 3, 3, 9]])
    P, M = lv.shape
    for mode in (0, 1):
        ctx = mc.Context([(L, P, 1, bs)])
        ctx.init_weights(lnW)
        tr_dev = ctx.new_trace(M)
        h = ctx.new_hist()
        ctx.run_chains(M, tr_dev, h)  # fills a real trace; replaced by the hand-built one below
        hand = torch.tensor(lv - N // 2, dtype=ctx.trace_dtype()).cuda()
        h.zero_()
        cut = ctx.new_cut()
        ctx.join(hand, cut, h, mode)
        ocut, oH, oret, osig = O.join(L, bs, 1, lv - N // 2, lnW, -1, 0, mode)
        assert np.array_equal(_np(cut), ocut)
        # the joint removed exactly the discarded configurations
        assert np.array_equal(-_np(h), np.bincount(lv.ravel(), minlength=N + 1) - oH)
        seam, rnd, _ = ctx.counters()
        assert seam == osig and rnd == 1
        ctx.close()
    assert list(ocut) == [1, 1, 1, 1]


def test_call_order_and_overflow_errors():
    mc = _mc()
    ctx = mc.Context([(8, 4, 1, 1)])
    tr = ctx.new_trace(10)
    h = ctx.new_hist()
    cut = ctx.new_cut()
    with pytest.raises(mc.MCError) as e:
        ctx.join(tr, cut, h)
    assert e.value.status == mc.MC_ESTATE
    ctx.run_chains(10, tr, h)
    with pytest.raises(mc.MCError) as e:
        ctx.join(ctx.new_trace(11), cut, h)
    assert e.value.status == mc.MC_EINVAL
    ctx.join(tr, cut, h)
    with pytest.raises(mc.MCError):
        ctx.init_weights(np.full(ctx.n_bins(), np.nan))
    # 2^20 chains x 4096 sweeps would overflow the int32 histogram: refused
    # before anything is launched
    import ctypes

    big = mc.Context([(8, 1 << 20, 1, 1)])
    tp = (ctypes.c_void_p * 1)(tr.data_ptr())
    hp = (ctypes.c_void_p * 1)(h.data_ptr())
    assert mc.lib().mc_run_chains(big._h, 4096, tp, hp) == mc.MC_EOVERFLOW
    ctx.close()
    big.close()


def test_bench_workload_full_size_sampled():
    """The L = 32 workload at full size (4096 chains, 10^5 sweeps, prior ln w)
    in its default launch configuration.  Sampled chains are replayed by the
    oracle bit for bit; the oracle redoes the whole joint over all 4096
    traces (every cut, the joined histogram, the seam and the retained count)
    and the weight update, which must agree exactly."""
    mc = _mc()
    L, P, M, N = 32, 4096, 100000, 1024
    w = _prior_lnW()
    ctx = mc.Context([(L, P, 1, 1)])
    ctx.init_weights(w)
    tr, h, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
    ctx.run_chains(M, tr, h)
    raw = _np(h).copy()
    ctx.join(tr, cut, h)
    joined = _np(h).copy()
    seam, rnd, sweep = ctx.counters()
    w2, flat, ret = ctx.update_weights(h)
    levels = ctx.levels()
    spins = {c: ctx.spins(c) for c in (0, 2047, 4095)}
    trace = _np(tr).astype(np.int32)
    del tr
    cuts = _np(cut)
    ctx.close()
    # sampled chains: the oracle replays them from their initial state
    for c in (0, 2047, 4095):
        s0 = O.init_chain(L, 1, c)
        m0 = (O.energy(L, s0) + 2 * N) // 4
        s, m, otr, _ = O.sweeps(L, 1, 1, c, s0, m0, 0, M, w)
        assert np.array_equal(trace[c], otr), c
        assert np.array_equal(spins[c], s) and levels[c] == m
    assert sweep == M and rnd == 1
    assert raw.sum() == P * M
    assert np.array_equal(raw, np.bincount(((trace + N // 2) >> 1).ravel(), minlength=513))
    # the whole joint and the update, recomputed by the oracle from the traces
    ocut, oH, oret, osig = O.join(L, 1, 1, trace, w, -1, 0)
    assert cuts[0] == 1  # the first chain of the first round has no seam
    assert np.array_equal(cuts, ocut)
    assert np.array_equal(joined, oH)
    assert seam == osig and ret == oret
    ow, oflat = O.update(L, 1, oH, w)
    assert flat == oflat
    assert np.array_equal(w2.view(np.uint64), ow.view(np.uint64))


@pytest.mark.parametrize("L,P,M,launch", [(128, 8192, 4, (32, 8)), (100, 8192, 4, (32, 8)), (256, 4096, 2, (16, 9))])
def test_large_workload_full_chain_count_sampled(L, P, M, launch):
    """The large-lattice workloads at their full chain counts in the default
    launch: L = 128 and the paper's L = 100 with 8192 chains (the quad
    streamed-row kernel, 32 chains on two consumer waves per workgroup, the
    per-bin table in LDS), L = 256 with 4096 chains (16 chains per workgroup,
    the per-bin table in global memory); a non-trivial weight (at ln w = 0
    every flip is accepted): sampled chains replayed by the oracle bit for
    bit; histograms and cut points through properties that hold at any
    size."""
    mc = _mc()
    N, bs = L * L, 1
    nb = (N >> bs) + 1
    w = _smooth_weight(L, bs, 21)
    ctx = mc.Context([(L, P, 1, bs)])
    ctx.init_weights(w)
    assert ctx.launch()[:2] == launch
    tr, h, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
    ctx.run_chains(M, tr, h)
    raw = _np(h).copy()
    ctx.join(tr, cut, h)
    joined = _np(h).copy()
    levels = ctx.levels()
    # 16: first chain of a workgroup's second consumer wave (32 per workgroup)
    sampled = (0, 15, 16, 31, 32, P // 2 - 1, P - 1)
    spins = {c: ctx.spins(c) for c in sampled}
    trace = _np(tr)
    cuts = _np(cut)
    ctx.close()
    for c in sampled:
        s0 = O.init_chain(L, 1, c)
        m0 = (O.energy(L, s0) + 2 * N) // 4
        s, m, otr, _ = O.sweeps(L, 1, bs, c, s0, m0, 0, M, w)
        assert np.array_equal(trace[c].astype(np.int32), otr), c
        assert np.array_equal(spins[c], s) and levels[c] == m, c
    lv = trace.astype(np.int64) + N // 2
    assert raw.sum() == P * M
    assert np.array_equal(raw, np.bincount((lv >> bs).ravel(), minlength=nb))
    keep = np.arange(M)[None, :] >= np.where(cuts > 0, cuts - 1, M)[:, None]
    assert np.array_equal(joined, np.bincount((lv[keep] >> bs), minlength=nb))
    sigma = -1
    for i in range(P):
        c = cuts[i]
        if sigma >= 0 and i % 61 == 0:
            ws = w[sigma >> bs]
            upto = (c - 1) if c > 0 else M
            for k in range(upto + (1 if c > 0 else 0)):
                acc = O.uniform(1, L, 2, 0, i, k) <= O.threshold(w[lv[i, k] >> bs] - ws)
                assert acc == (c > 0 and k == c - 1), (i, k, c)
        if c > 0:
            sigma = int(lv[i, M - 1])


def test_batched_workload_full_chain_count_sampled():
    """The batched workload's sizes and chain counts (L = 16, 24, 32, 48, 64,
    2048 chains each) in one persistent launch in the autotuned plans the
    benchmark times, with non-trivial weights:
    sampled chains of every size replayed by the oracle, raw histograms equal
    to the bincount of the traces."""
    mc = _mc()
    Ls, P, M, bs = [16, 24, 32, 48, 64], 2048, 12, 1
    ws = [_smooth_weight(L, bs, 30 + L) for L in Ls]
    ctx = mc.Context([(L, P, 1, bs) for L in Ls])
    for i, w in enumerate(ws):
        ctx.init_weights(w, i)
    ctx.autotune(200)  # as the benchmark does; its probes leave the chains untouched
    assert all(ctx.launch(i)[2] for i in range(len(Ls)))  # batched
    trs = [ctx.new_trace(M, i) for i in range(len(Ls))]
    hs = [ctx.new_hist(i) for i in range(len(Ls))]
    ctx.run_chains(M, trs, hs)
    sampled = (0, 63, 64, 1023, 2047)
    res = []
    for i, L in enumerate(Ls):
        res.append((_np(trs[i]), _np(hs[i]).copy(), ctx.levels(i), {c: ctx.spins(c, i) for c in sampled}))
    ctx.close()
    for i, L in enumerate(Ls):
        N = L * L
        trace, raw, levels, spins = res[i]
        for c in sampled:
            s0 = O.init_chain(L, 1, c)
            m0 = (O.energy(L, s0) + 2 * N) // 4
            s, m, otr, _ = O.sweeps(L, 1, bs, c, s0, m0, 0, M, ws[i])
            assert np.array_equal(trace[c].astype(np.int32), otr), (L, c)
            assert np.array_equal(spins[c], s) and levels[c] == m, (L, c)
        lv = trace.astype(np.int64) + N // 2
        assert np.array_equal(raw, np.bincount((lv >> bs).ravel(), minlength=(N >> bs) + 1)), L


@pytest.mark.parametrize("cpb,kind", [(16, 7), (64, 4)])
@pytest.mark.parametrize("L,P,bs,M", [(8, 37, 1, 20), (12, 20, 0, 12), (16, 33, 1, 10), (32, 70, 1, 4),
                                      (48, 17, 1, 3), (64, 21, 1, 2)])
def test_producer_consumer_kernels_bitexact(L, P, bs, M, cpb, kind):
    """The quad-speculative kernel (kind 7: four lanes per chain, four sites per
    step; 16 chains per workgroup, the default) and the pair kernel (kind 4:
    one lane per chain, chosen with more chains per workgroup than kind 7
    takes), against the oracle over two rounds with ragged workgroups."""
    mc = _mc()
    w = _smooth_weight(L, bs, 40 + L)
    ctx = mc.Context([(L, P, 2, bs)])
    ctx.init_weights(w)
    ctx.set_chains_per_block(cpb)
    assert ctx.launch()[1] == kind, ctx.launch()
    R = O.Run(L, P, seed=2, bin_shift=bs, lnW=w)
    for _ in range(2):
        g = gpu_round(ctx, M)
        o = oracle_round(R, M)
        assert_round_equal(g, o)
    assert_state_equal(ctx, R)
    ctx.close()


def test_set_launch_kinds_and_refusals():
    """mc_set_launch picks a kind other than the default at the same chains
    per workgroup (the pair kernel and a one-wave kernel at 16 chains, where
    mc_set_chains_per_block takes the quad kernel), with the same results as
    the oracle; a kind that cannot run the size there, a kind out of range or
    a chains-per-workgroup count out of range is refused and changes
    nothing."""
    mc = _mc()
    L, P, bs, M = 16, 40, 1, 8
    w = _smooth_weight(L, bs, 77)
    for kind in (4, 0):
        ctx = mc.Context([(L, P, 2, bs)])
        ctx.init_weights(w)
        ctx.set_launch(kind, 16)
        assert ctx.launch()[:2] == (16, kind)
        R = O.Run(L, P, seed=2, bin_shift=bs, lnW=w)
        g = gpu_round(ctx, M)
        o = oracle_round(R, M)
        assert_round_equal(g, o)
        ctx.close()
    ctx = mc.Context([(32, 20, 1, 1), (128, 20, 1, 1)])
    before = ctx.launch(0), ctx.launch(1)
    for i, kind, cpb in ((0, 7, 17), (0, 8, 16), (1, 7, 16), (0, 10, 16), (0, 7, 0), (1, 8, 33)):
        with pytest.raises(mc.MCError) as e:
            ctx.set_launch(kind, cpb, i)
        assert e.value.status == mc.MC_EINVAL, (i, kind, cpb)
    assert (ctx.launch(0), ctx.launch(1)) == before
    ctx.set_launch(7, 8, 0)
    assert ctx.launch(0)[:2] == (8, 7)
    ctx.close()


@pytest.mark.parametrize("L,P,kinds", [(16, 45, (0, 1, 2, 4, 7)), (64, 19, (0, 1, 2, 4, 7)),
                                       (128, 40, (5, 6, 8, 9)), (100, 21, (8, 9))])
def test_every_kernel_kind_bitexact(L, P, kinds):
    """Every kernel kind that runs a size, set with mc_set_launch (the one-wave
    kinds with the thresholds in LDS (0) or global memory (1), the lattice in
    global memory (2), the pair (4) and quad (7) kernels; at the large sizes
    the one-lane (5, 6) and quad (8, 9) streamed-row kernels with the table in
    LDS or global memory), against the oracle over two rounds with a ragged
    last workgroup."""
    mc = _mc()
    bs, M = 1, 3
    w = _smooth_weight(L, bs, 90 + L)
    for kind in kinds:
        cpb = 16 if kind in (0, 1, 2, 4, 7, 9) else 32
        ctx = mc.Context([(L, P, 4, bs)])
        ctx.init_weights(w)
        ctx.set_launch(kind, cpb)
        assert ctx.launch()[:2] == (cpb, kind), (kind, ctx.launch())
        R = O.Run(L, P, seed=4, bin_shift=bs, lnW=w)
        for _ in range(2):
            g = gpu_round(ctx, M)
            o = oracle_round(R, M)
            assert_round_equal(g, o)
        assert_state_equal(ctx, R)
        ctx.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_one_sweep_rounds_bitexact(mode):
    """Rounds of a single sweep (every trace holds one configuration, so each
    cut point is 1 or -1) on the quad kernel, four rounds with an update after
    each, in every joint mode (detailed balance in chain order, naive splice,
    detailed balance in energy order), against the oracle."""
    mc = _mc()
    L, P, bs = 16, 50, 1
    w = _smooth_weight(L, bs, 61)
    ctx = mc.Context([(L, P, 6, bs)])
    ctx.init_weights(w)
    assert ctx.launch()[1] == 7
    R = O.Run(L, P, seed=6, bin_shift=bs, lnW=w)
    for _ in range(4):
        g = gpu_round(ctx, 1, mode=mode)
        o = oracle_round(R, 1, mode=mode)
        assert_round_equal(g, o)
        assert set(np.unique(g["cut"]).tolist()) <= {-1, 1}
    assert_state_equal(ctx, R)
    ctx.close()


@pytest.mark.parametrize("L,kind", [(32, 7), (128, 8)])
def test_single_chain_bitexact(L, kind):
    """One chain: a workgroup with one of its 16 (or 32) chain slots used, and
    joints that only ever test the chain against its own previous seam; three
    rounds with updates in chain and energy order, against the oracle."""
    mc = _mc()
    bs = 1
    w = _smooth_weight(L, bs, 62)
    for mode in (0, 2):
        ctx = mc.Context([(L, 1, 8, bs)])
        ctx.init_weights(w)
        assert ctx.launch()[1] == kind
        R = O.Run(L, 1, seed=8, bin_shift=bs, lnW=w)
        for _ in range(3):
            g = gpu_round(ctx, 5, mode=mode)
            o = oracle_round(R, 5, mode=mode)
            assert_round_equal(g, o)
        assert_state_equal(ctx, R)
        ctx.close()
