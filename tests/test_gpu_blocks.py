"""A run split into blocks of chains, as over several GPUs (the exchange of
the sharding design, on one device): contexts holding chains 0 .. p/2-1 and
p/2 .. p-1 (chain_offset) make the traces of one context holding all p; their
joints, taken in turn with the seam handed on (mc_get_counters /
mc_set_seam), keep what the one joint keeps; and the sum of their histograms
(the all-reduce) gives every block the whole run's weight update.  Bit for
bit, over three iterations."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,P,bs", [(32, 200, 1), (128, 40, 1)])
def test_split_run_equals_whole_run(L, P, bs):
    import paper_0812_2964_amd as mc

    M = 30
    nb = ((L * L) >> bs) + 1
    x = (np.arange(nb) - nb / 2) / nb
    w = -0.4 * L * L * x * x + np.random.default_rng(3).normal(0, 0.5, nb)
    whole = mc.Context([(L, P, 5, bs)])
    blocks = [mc.Context([(L, P // 2, 5, bs, 0)]), mc.Context([(L, P // 2, 5, bs, P // 2)])]
    for c in [whole] + blocks:
        c.init_weights(w)
    for it in range(3):
        tr, h, cut = whole.new_trace(M), whole.new_hist(), whole.new_cut()
        whole.run_chains(M, tr, h)
        whole.join(tr, cut, h)
        bt = [b.new_trace(M) for b in blocks]
        bh = [b.new_hist() for b in blocks]
        bc = [b.new_cut() for b in blocks]
        for b, t, hh in zip(blocks, bt, bh):
            b.run_chains(M, t, hh)
        assert np.array_equal(np.concatenate([t.cpu().numpy() for t in bt]), tr.cpu().numpy()), it
        # the ring of Algorithm step 4: the first block starts where the last one ended
        blocks[0].set_seam(blocks[1].counters()[0])
        blocks[0].join(bt[0], bc[0], bh[0])
        blocks[1].set_seam(blocks[0].counters()[0])
        blocks[1].join(bt[1], bc[1], bh[1])
        assert np.array_equal(np.concatenate([c.cpu().numpy() for c in bc]), cut.cpu().numpy()), it
        hsum = bh[0] + bh[1]
        assert np.array_equal(hsum.cpu().numpy(), h.cpu().numpy()), it
        assert blocks[1].counters()[0] == whole.counters()[0]
        ww, fw, _ = whole.update_weights(h)
        for b in blocks:
            wb, fb, _ = b.update_weights(hsum.clone())
            assert np.array_equal(wb.view(np.uint64), ww.view(np.uint64)) and fb == fw, it
    for c in [whole] + blocks:
        c.close()


@pytest.mark.parametrize("sizes", [[(32, 300, 2, 1)], [(128, 70, 2, 1)], [(16, 100, 2, 1), (64, 50, 2, 1)]])
def test_runs_are_deterministic(sizes):
    """The same run twice in fresh contexts gives the same bits: traces, cuts,
    joined histograms (LDS histograms merged with atomics, the speculative
    joint) and ln w, for the quad kernels of both lattice ranges and the
    batched launch."""
    import paper_0812_2964_amd as mc

    def run():
        ctx = mc.Context(sizes)
        out = []
        for _ in range(2):
            trs = [ctx.new_trace(40, i) for i in range(len(sizes))]
            hs = [ctx.new_hist(i) for i in range(len(sizes))]
            cuts = [ctx.new_cut(i) for i in range(len(sizes))]
            ctx.run_chains(40, trs, hs)
            for i in range(len(sizes)):
                ctx.join(trs[i], cuts[i], hs[i], i=i)
                joined = hs[i].cpu().numpy().copy()
                w, _, _ = ctx.update_weights(hs[i], i=i)
                out.append((trs[i].cpu().numpy(), cuts[i].cpu().numpy(), joined, w.view(np.uint64)))
        ctx.close()
        return out

    a, b = run(), run()
    for xa, xb in zip(a, b):
        for ya, yb in zip(xa, xb):
            assert np.array_equal(ya, yb)
