"""Batched sizes in one persistent launch, graph-captured recursion, launch
configuration: none of them may change a single bit of the results.

* every size of a batched context equals the same size run alone, and the
  oracle, bit for bit (a chain's random words are keyed by its own size and
  index, so batching cannot change its trajectory);
* a captured graph of whole iterations, replayed several times with eager
  work and synchronisations in between, equals the same iterations issued one
  call at a time;
* any chains-per-workgroup setting and the autotuner's choice give the same
  bits.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

SIZES = [(16, 70, 1, 1), (24, 33, 1, 1), (32, 65, 1, 1), (48, 20, 1, 1), (64, 17, 1, 1)]


def _mc():
    import paper_0812_2964_amd as mc

    return mc


def _np(t):
    return t.detach().cpu().numpy()


def _weights(L, bs, seed):
    N = L * L
    nb = (N >> bs) + 1
    x = (np.arange(nb) - nb / 2) / nb
    return -0.2 * N * x * x + np.random.default_rng(seed).normal(0, 0.3, nb)


def _iterate(ctx, M, n_iter):
    """n_iter eager iterations of every size; returns per-size lists of
    (trace, cut, joined hist, ln w)."""
    n = len(ctx.sizes)
    out = [[] for _ in range(n)]
    for _ in range(n_iter):
        trs = [ctx.new_trace(M, i) for i in range(n)]
        hs = [ctx.new_hist(i) for i in range(n)]
        ctx.run_chains(M, trs, hs)
        for i in range(n):
            cut = ctx.new_cut(i)
            ctx.join(trs[i], cut, hs[i], 0, i)
            joined = _np(hs[i]).copy()
            w, _, _ = ctx.update_weights(hs[i], i)
            out[i].append((_np(trs[i]).astype(np.int32), _np(cut), joined, w))
    return out


def test_batched_equals_standalone_and_oracle():
    mc = _mc()
    M, n_iter = 12, 2
    ctx = mc.Context(SIZES)
    for i, (L, P, seed, bs) in enumerate(SIZES):
        ctx.init_weights(_weights(L, bs, L), i)
    assert all(ctx.launch(i)[2] for i in range(len(SIZES)))  # one persistent launch
    got = _iterate(ctx, M, n_iter)
    for i, (L, P, seed, bs) in enumerate(SIZES):
        alone = mc.Context([(L, P, seed, bs)])
        alone.init_weights(_weights(L, bs, L))
        ref = _iterate(alone, M, n_iter)[0]
        R = O.Run(L, P, seed=seed, bin_shift=bs, lnW=_weights(L, bs, L))
        for it in range(n_iter):
            tr, cut, H, w = got[i][it]
            assert np.array_equal(tr, ref[it][0]) and np.array_equal(cut, ref[it][1])
            assert np.array_equal(H, ref[it][2])
            assert np.array_equal(w.view(np.uint64), ref[it][3].view(np.uint64))
            otr, _ = R.run(M)
            ocut, _ = R.join(otr)
            oH = R.H.copy()
            R.update()
            assert np.array_equal(tr, otr), (L, it)
            assert np.array_equal(cut, ocut) and np.array_equal(H, oH)
            assert np.array_equal(w.view(np.uint64), R.lnW.view(np.uint64))
        alone.close()
    ctx.close()


def test_graph_replays_equal_eager_iterations():
    mc = _mc()
    M, per_graph, replays = 10, 3, 2
    eager = mc.Context(SIZES)
    graph_ctx = mc.Context(SIZES)
    for i, (L, P, seed, bs) in enumerate(SIZES):
        eager.init_weights(_weights(L, bs, L + 1), i)
        graph_ctx.init_weights(_weights(L, bs, L + 1), i)
    n = len(SIZES)
    trs = [graph_ctx.new_trace(M, i) for i in range(n)]
    hs = [graph_ctx.new_hist(i) for i in range(n)]
    cuts = [graph_ctx.new_cut(i) for i in range(n)]
    g = graph_ctx.graph(M, per_graph, trs, hs, cuts)
    for rep in range(replays):
        ref = _iterate(eager, M, per_graph)  # eager work between the replays
        g.launch()
        graph_ctx.sync()
        for i in range(n):
            tr_last, cut_last, _, w_last = ref[i][-1]
            assert np.array_equal(_np(trs[i]).astype(np.int32), tr_last), (rep, i)
            assert np.array_equal(_np(cuts[i]), cut_last)
            assert np.array_equal(graph_ctx.weights(i).view(np.uint64), w_last.view(np.uint64))
            assert not _np(hs[i]).any()
            updates, _, _, _ = graph_ctx.progress(i)
            assert updates == per_graph * (rep + 1)
            assert graph_ctx.counters(i) == eager.counters(i)
    with pytest.raises(mc.MCError):
        graph_ctx.set_chains_per_block(16, 0)  # fixed while a graph exists
    g.close()
    graph_ctx.close()
    eager.close()


def test_twenty_iteration_graph_of_the_batched_workload():
    """The batched workload's five sizes at their full chain counts (2048
    each), the recursion's first 20 iterations captured in ONE graph (at 20
    sweeps per iteration instead of 10^5), equal 20 eager iterations bit for
    bit: weights, counters, progress, the last iteration's traces and cuts."""
    mc = _mc()
    Ls, P, M, n_it = [16, 24, 32, 48, 64], 2048, 20, 20
    sizes = [(L, P, 1, 1) for L in Ls]
    g_ctx = mc.Context(sizes)
    e_ctx = mc.Context(sizes)
    n = len(Ls)
    trs = [g_ctx.new_trace(M, i) for i in range(n)]
    hs = [g_ctx.new_hist(i) for i in range(n)]
    cuts = [g_ctx.new_cut(i) for i in range(n)]
    g = g_ctx.graph(M, n_it, trs, hs, cuts)
    g.launch()
    g_ctx.sync()
    ref = _iterate(e_ctx, M, n_it)
    for i in range(n):
        tr_last, cut_last, _, w_last = ref[i][-1]
        assert np.array_equal(_np(trs[i]).astype(np.int32), tr_last), Ls[i]
        assert np.array_equal(_np(cuts[i]), cut_last), Ls[i]
        assert np.array_equal(g_ctx.weights(i).view(np.uint64), w_last.view(np.uint64)), Ls[i]
        assert g_ctx.progress(i) == e_ctx.progress(i) and g_ctx.progress(i)[0] == n_it
        assert g_ctx.counters(i) == e_ctx.counters(i)
    g.close()
    g_ctx.close()
    e_ctx.close()


def test_launch_configuration_never_changes_results():
    mc = _mc()
    M = 15
    ref = None
    for cpb in (None, 1, 13, 32, 64, "auto"):
        ctx = mc.Context(SIZES[:3])
        for i, (L, P, seed, bs) in enumerate(SIZES[:3]):
            ctx.init_weights(_weights(L, bs, 7), i)
        if cpb == "auto":
            chosen = ctx.autotune(5)
            assert all(c in (16, 32, 64) for c in chosen)
            assert [ctx.counters(i)[2] for i in range(3)] == [0, 0, 0]  # probes left the chains alone
        elif cpb is not None:
            for i in range(3):
                ctx.set_chains_per_block(cpb, i)
        res = _iterate(ctx, M, 1)
        flat = [np.concatenate([r[0][0].ravel(), r[0][1], r[0][2]]) for r in res]
        if ref is None:
            ref = flat
        else:
            for a, b in zip(flat, ref):
                assert np.array_equal(a, b), cpb
        ctx.close()
