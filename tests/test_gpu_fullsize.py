"""The largest workloads at their full size, element by element against the
oracle where the oracle can afford it.

- L = 128, 8192 chains, one whole iteration of 2 x 10^5 sweeps (Algorithm
  step 2), the joint of steps 3-5 and the update of eq. (new_weight) (the
  large-lattice recursion's per-iteration work).  The sweeps run as four
  launches of one round (mc_run_chains_part), so that progress is reported
  between them; parts equal one launch bit for bit (tested elsewhere).  Two
  sampled chains are replayed by the oracle over all 2 x 10^5 sweeps while the
  GPU runs; the oracle recomputes the whole joint over all 8192 traces and the
  update, and cuts, joined histogram, seam, retained count, flatness and ln w
  must agree exactly.  The weight is a smooth non-trivial one (from ln w = 0
  every move is accepted and the trace is constant, which would test little).
- The learned initialiser's prediction at L = 256 (32769 bins) against the
  fp64 network oracle, and 4096 chains of L = 256 initialised with it, sampled
  chains replayed by the oracle.
"""
import threading
import time

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def _weight(L, bs, seed, amp):
    rng = np.random.default_rng(seed)
    nb = ((L * L) >> bs) + 1
    x = (np.arange(nb) - nb / 2) / nb
    return -0.5 * L * L * x * x + rng.normal(0, amp, nb)


def test_large_lattice_full_iteration(capsys):
    import paper_0812_2964_amd as mc
    import torch

    L, P, M, bs = 128, 8192, 200000, 1
    N = L * L
    parts = 4
    t0 = time.perf_counter()

    def say(msg):
        with capsys.disabled():
            print("  L=128 full iteration: %s (%.0f s)" % (msg, time.perf_counter() - t0), flush=True)

    w = _weight(L, bs, 128, 1.5)
    ctx = mc.Context([(L, P, 1, bs)])
    assert ctx.launch()[1] == 8
    ctx.init_weights(w)
    # the oracle replays two chains (the first, and the last of the second
    # consumer wave of a workgroup) on host threads while the GPU sweeps
    sample = [0, 31 + 32 * 97]
    replay = {}

    def oracle_chain(c):
        s0 = O.init_chain(L, 1, c)
        m0 = (O.energy(L, s0) + 2 * N) // 4
        replay[c] = O.sweeps(L, 1, bs, c, s0, m0, 0, M, w)

    threads = [threading.Thread(target=oracle_chain, args=(c,)) for c in sample]
    for th in threads:
        th.start()
    tr, h, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
    for k in range(parts):
        ctx.run_chains_part(M // parts, k * (M // parts), tr, h)
        ctx.sync()
        say("sweeps %d of %d done" % ((k + 1) * (M // parts), M))
    raw = h.cpu().numpy().copy()
    ctx.join(tr, cut, h)
    joined = h.cpu().numpy().copy()
    gcut = cut.cpu().numpy()
    w2, flat, ret = ctx.update_weights(h)
    seam = ctx.counters()[0]
    levels = ctx.levels()
    spins = {c: ctx.spins(c) for c in sample}
    trace = tr.cpu().numpy()
    del tr
    torch.cuda.synchronize()
    ctx.close()
    say("joint and update done")
    assert raw.sum() == P * M
    tr32 = trace.astype(np.int32)
    del trace
    ocut, oH, oret, osig = O.join(L, bs, 1, tr32, w, -1, 0)
    say("oracle joint done")
    assert np.array_equal(gcut, ocut)
    assert np.array_equal(joined, oH)
    assert ret == oret and seam == osig
    assert np.array_equal(raw, np.bincount((tr32.ravel() + N // 2) >> bs, minlength=(N >> bs) + 1))
    ow, oflat = O.update(L, bs, oH, w)
    assert flat == oflat
    assert np.array_equal(w2.view(np.uint64), ow.view(np.uint64))
    for th in threads:
        th.join()
    say("oracle replays done")
    for c in sample:
        s, m, otr, _ = replay[c]
        assert np.array_equal(tr32[c], otr), c
        assert np.array_equal(spins[c], s) and levels[c] == m, c


def test_learned_prediction_and_initialisation_at_L256():
    import paper_0812_2964_amd as mc

    L, bs = 256, 1
    N = L * L
    nb = (N >> bs) + 1
    rng = np.random.default_rng(256)
    params = rng.normal(0, 0.3, O.mlp_n_params()).astype(np.float32)
    net = mc.MLP(params=params)
    pw = net.predict_weights(L, bs)
    assert pw.shape == (nb,) and np.isfinite(pw).all()
    e = ((4.0 * (2 * np.arange(nb) + 0.5) - 2 * N) / N).astype(np.float32)
    x = np.column_stack([np.full(nb, np.float32(1.0 / L)), e]).astype(np.float64)
    want = -N * O.mlp_forward(params.astype(np.float64), x)
    # fp32 network: relative error of a few 2^-24 per layer, times N
    assert np.abs(pw - want).max() <= 3e-5 * N
    # 4096 chains of L = 256 start from the proposal (the large lattice's
    # initial weight), sampled chains against the oracle
    P, M = 4096, 2
    ctx = mc.Context([(L, P, 1, bs)])
    ctx.init_weights(pw)
    tr, h = ctx.new_trace(M), ctx.new_hist()
    ctx.run_chains(M, tr, h)
    trace = tr.cpu().numpy().astype(np.int32)
    assert h.cpu().numpy().sum() == P * M
    for c in (0, 15, 16, 2047, 4095):
        s0 = O.init_chain(L, 1, c)
        m0 = (O.energy(L, s0) + 2 * N) // 4
        _, _, otr, _ = O.sweeps(L, 1, bs, c, s0, m0, 0, M, pw)
        assert np.array_equal(trace[c], otr), c
    ctx.close()


def test_batched_workload_two_iterations_as_benchmarked(capsys):
    """The batched workload exactly as the benchmark times it: L = 16, 24,
    32, 48, 64 with 2048 chains each, autotuned, one HIP graph of a whole
    iteration (10^5 sweeps of every chain in one persistent launch, the
    joints and the updates) replayed twice from ln w = 0.  For every size the
    oracle redoes both joints over all 2048 traces (cut points exactly) and
    both updates (ln w bit for bit, which pins each joined histogram, since
    ln is one-to-one on the counts), and replays sampled chains over both
    iterations, the second under the first update's weight."""
    import paper_0812_2964_amd as mc
    from concurrent.futures import ThreadPoolExecutor

    Ls, P, M, bs = [16, 24, 32, 48, 64], 2048, 100000, 1
    sample = (0, 1001, 2047)
    t0 = time.perf_counter()

    def say(msg):
        with capsys.disabled():
            print("  batched, two iterations: %s (%.0f s)" % (msg, time.perf_counter() - t0), flush=True)

    ctx = mc.Context([(L, P, 1, bs) for L in Ls])
    ctx.autotune(200)
    assert all(ctx.launch(i)[2] for i in range(len(Ls)))  # one batched launch
    trs = [ctx.new_trace(M, i) for i in range(len(Ls))]
    hs = [ctx.new_hist(i) for i in range(len(Ls))]
    cuts = [ctx.new_cut(i) for i in range(len(Ls))]
    g = ctx.graph(M, 1, trs, hs, cuts)
    got = []  # per iteration: per size (trace int16, cuts, ln w, flat, seam)
    pool = ThreadPoolExecutor(max_workers=8)

    def replay(L, c, s, m, g0, w):
        return O.sweeps(L, 1, bs, c, s, m, g0, M, w)

    # iteration 1 from ln w = 0: the oracle's replays run while the GPU sweeps
    first = {}
    for L in Ls:
        N = L * L
        for c in sample:
            s0 = O.init_chain(L, 1, c)
            first[(L, c)] = pool.submit(replay, L, c, s0, (O.energy(L, s0) + 2 * N) // 4, 0,
                                        np.zeros((N >> bs) + 1))
    for it in range(2):
        g.launch()
        ctx.sync()
        got.append([(trs[i].cpu().numpy(), cuts[i].cpu().numpy(), ctx.weights(i), ctx.progress(i)[2],
                     ctx.counters(i)[0]) for i in range(len(Ls))])
        say("iteration %d on the GPU done" % (it + 1))
    levels = [ctx.levels(i) for i in range(len(Ls))]
    spins = [{c: ctx.spins(c, i) for c in sample} for i in range(len(Ls))]
    g.close()
    ctx.close()
    second = {}
    for i, L in enumerate(Ls):
        N = L * L
        w, seam = np.zeros((N >> bs) + 1), -1
        for it in range(2):
            tr, gcut, gw, gflat, gseam = got[it][i]
            tr32 = tr.astype(np.int32)
            ocut, oH, oret, osig = O.join(L, bs, 1, tr32, w, seam, it)
            assert np.array_equal(gcut, ocut), (L, it)
            assert gseam == osig, (L, it)
            ow, oflat = O.update(L, bs, oH, w)
            assert gflat == oflat, (L, it)
            assert np.array_equal(gw.view(np.uint64), ow.view(np.uint64)), (L, it)
            if it == 0:
                for c in sample:
                    s, m, otr, _ = first[(L, c)].result()
                    assert np.array_equal(tr32[c], otr), (L, c, it)
                    second[(L, c)] = pool.submit(replay, L, c, s, m, M, ow)
            w, seam = ow, osig
            del tr32
        say("oracle joints and updates of L = %d done" % L)
    for i, L in enumerate(Ls):
        tr32 = got[1][i][0].astype(np.int32)
        for c in sample:
            s, m, otr, _ = second[(L, c)].result()
            assert np.array_equal(tr32[c], otr), (L, c, 1)
            assert np.array_equal(spins[i][c], s) and levels[i][c] == m, (L, c)
    pool.shutdown()
    say("oracle replays done")
