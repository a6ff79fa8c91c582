"""Learned initial weights for the multicanonical recursion.

The recursion of Sec. 3.1 (w <- w/h) extends the sampled energy range by
roughly ln(samples per iteration) of ln g per iteration, so from w = 1 it
needs many iterations on large lattices.  The entropy per site s(e) = ln g/N
depends on the lattice size only through small finite-size terms, so a network
trained on the converged weights of small lattices proposes a weight for a
larger one; the recursion then continues from there, and w = 1 stays the
fallback.  Every step runs in the library's kernels (recursion, target
construction, training, prediction); this module only sequences the calls.
"""
import numpy as np

from . import Context, MLP, mlp_targets


def run_to_flat(L, n_chains, n_sweeps, cap, lnW0=None, seed=1, bin_shift=1, extra=0, per_launch=4, progress=None):
    """Recursion until the first flat histogram (then `extra` more
    iterations), at most `cap` iterations, replaying a captured graph of
    `per_launch` iterations.  progress(iterations done), if given, is called
    after every replay.  Returns (ln w, first flat iteration or None,
    iterations run)."""
    ctx = Context([(L, n_chains, seed, bin_shift)])
    ctx.init_weights(lnW0)
    trace, hist, cut = ctx.new_trace(n_sweeps), ctx.new_hist(), ctx.new_cut()
    graph = ctx.graph(n_sweeps, per_launch, [trace], [hist], [cut])
    done, flat_at = 0, None
    while done < cap:
        graph.launch()
        done += per_launch
        updates, first_flat, _, _ = ctx.progress()
        if progress is not None:
            progress(done)
        if first_flat and flat_at is None:
            flat_at = first_flat
        if flat_at is not None and updates >= flat_at + extra:
            break
    ctx.sync()
    lnW = ctx.weights()
    graph.close()
    ctx.close()
    return lnW, flat_at, done


class Initializer:
    """The network and its training data: converged ln w of several sizes."""

    def __init__(self, seed=1):
        import torch

        self.mlp = MLP(seed=seed)
        self.xs, self.ts, self.ws = [], [], []
        self._torch = torch

    def add(self, L, lnW, bin_shift=1):
        x, t = mlp_targets(lnW, L, bin_shift)
        # each lattice size weighs the same in the loss
        w = self._torch.full((t.numel(),), 1.0 / t.numel(), dtype=self._torch.float32, device="cuda")
        self.xs.append(x)
        self.ts.append(t)
        self.ws.append(w)

    def fit(self, steps=4000, lr=2e-3):
        x = self._torch.cat(self.xs).contiguous()
        t = self._torch.cat(self.ts).contiguous()
        w = self._torch.cat(self.ws).contiguous()
        return self.mlp.train(x, t, w, steps=steps, lr=lr)

    def predict(self, L, bin_shift=1):
        return self.mlp.predict_weights(L, bin_shift)


def relative_spread(lnW_a, lnW_b):
    """max - min of the difference of two ln w (equal up to a constant = 0)."""
    d = np.asarray(lnW_a) - np.asarray(lnW_b)
    return float(d.max() - d.min())
