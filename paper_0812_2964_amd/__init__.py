"""Python binding of libmcgpu.so, the MI355X (gfx950) implementation of the
parallel multicanonical Markov-chain method of arXiv 0812.2964 (Sugihara,
Higo, Nakamura) on the periodic 2D Ising model.

This module only marshals arguments: every step of the method runs in the
library's HIP kernels.  PyTorch provides device memory (traces, histograms,
cut arrays are torch tensors) and the HIP stream.  There is no CPU fallback:
if the library is missing or no GPU is present, the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcgpu.so")

MC_OK, MC_EINVAL, MC_ENOMEM, MC_ENODEV, MC_EHIP, MC_ESTATE, MC_EOVERFLOW, MC_ECORRUPT, MC_EINTERNAL = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
_STATUS = {0: "MC_OK", -1: "MC_EINVAL", -2: "MC_ENOMEM", -3: "MC_ENODEV", -4: "MC_EHIP", -5: "MC_ESTATE",
           -6: "MC_EOVERFLOW", -7: "MC_ECORRUPT", -8: "MC_EINTERNAL"}

# Symbols declared in include/mc.h (checked by the CPU test-suite).
EXPORTED = ["mc_create", "mc_destroy", "mc_n_bins", "mc_trace_elem_bytes", "mc_lattice_words", "mc_init_weights",
            "mc_run_chains", "mc_join", "mc_update_weights", "mc_get_levels", "mc_get_lattice", "mc_get_counters",
            "mc_get_weights", "mc_get_progress", "mc_set_chains_per_block", "mc_set_launch", "mc_get_launch", "mc_autotune",
            "mc_graph_create", "mc_graph_launch", "mc_graph_destroy", "mc_sync", "mc_last_error",
            "mc_mlp_n_params", "mc_mlp_workspace_bytes", "mc_mlp_init", "mc_mlp_forward", "mc_mlp_loss_grad",
            "mc_mlp_train", "mc_mlp_targets", "mc_mlp_predict_weights", "mc_thermo", "mc_iterate_topup",
            "mc_get_state", "mc_set_state", "mc_set_seam", "mc_run_chains_part", "mc_get_stats", "mc_check_levels",
            "mc_probe", "mc_thermo_static"]


class MCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class Stats(ctypes.Structure):
    """mc_stats: progress, the last update's histogram and ln w range, the
    last joint's cut statistics and the device counters of one size."""
    _fields_ = [("updates", ctypes.c_int32), ("first_flat", ctypes.c_int32), ("last_flat", ctypes.c_int32),
                ("n_reach_bins", ctypes.c_int32), ("retained_last", ctypes.c_int64), ("hist_sum", ctypes.c_int64),
                ("hist_min", ctypes.c_int64), ("lnw_min", ctypes.c_double), ("lnw_max", ctypes.c_double),
                ("join_none", ctypes.c_int32), ("join_cut_max", ctypes.c_int32), ("join_cut_sum", ctypes.c_int64),
                ("sweep_index", ctypes.c_uint32), ("round_index", ctypes.c_uint32), ("seam", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class _Size(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("n_chains", ctypes.c_int32), ("seed", ctypes.c_uint32),
                ("bin_shift", ctypes.c_int32), ("chain_offset", ctypes.c_uint32)]


_lib = None


def lib():
    """Load the HIP library (after torch, so one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmcgpu.so is not built: run python -m paper_0812_2964_amd.build")
    import torch  # noqa: F401  (loads the HIP runtime the library links against)

    L = ctypes.CDLL(LIB_PATH)
    p, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    L.mc_create.argtypes = [ctypes.POINTER(_Size), i32, p, ctypes.POINTER(p)]
    L.mc_destroy.argtypes = [p]
    for f in ("mc_n_bins", "mc_trace_elem_bytes", "mc_lattice_words"):
        getattr(L, f).argtypes = [p, i32]
        getattr(L, f).restype = i32
    L.mc_init_weights.argtypes = [p, i32, p, i32]
    L.mc_run_chains.argtypes = [p, i64, p, p]
    L.mc_run_chains_part.argtypes = [p, i64, i64, i64, p, p]
    L.mc_get_stats.argtypes = [p, i32, ctypes.POINTER(Stats)]
    L.mc_check_levels.argtypes = [p, i32, ctypes.POINTER(i64)]
    L.mc_probe.argtypes = [i32, i32, p, p]
    L.mc_thermo_static.argtypes = [p, i32, p, i32, p]
    L.mc_join.argtypes = [p, i32, p, i64, p, p, i32]
    L.mc_update_weights.argtypes = [p, i32, p, p, p, p]
    L.mc_iterate_topup.argtypes = [p, i64, i64, i32, p, p, p, i32, p, p, p, p]
    L.mc_get_state.argtypes = [p, p, ctypes.POINTER(ctypes.c_size_t)]
    L.mc_set_seam.argtypes = [p, i32, i32]
    L.mc_set_state.argtypes = [p, p, ctypes.c_size_t]
    L.mc_get_levels.argtypes = [p, i32, p]
    L.mc_get_lattice.argtypes = [p, i32, i32, p, i32]
    L.mc_get_counters.argtypes = [p, i32, p, p, p]
    L.mc_get_weights.argtypes = [p, i32, p, i32]
    L.mc_get_progress.argtypes = [p, i32, p, p, p, p]
    L.mc_set_chains_per_block.argtypes = [p, i32, i32]
    L.mc_set_launch.argtypes = [p, i32, i32, i32]
    L.mc_get_launch.argtypes = [p, i32, p, p, p]
    L.mc_autotune.argtypes = [p, i64, p]
    L.mc_graph_create.argtypes = [p, i64, i32, p, p, p, i32, ctypes.POINTER(p)]
    L.mc_graph_launch.argtypes = [p, p]
    L.mc_graph_destroy.argtypes = [p]
    L.mc_sync.argtypes = [p]
    L.mc_last_error.restype = ctypes.c_char_p
    L.mc_mlp_n_params.restype = i32
    L.mc_mlp_workspace_bytes.argtypes = [i32]
    L.mc_mlp_workspace_bytes.restype = ctypes.c_size_t
    L.mc_mlp_init.argtypes = [p, u32, p]
    L.mc_mlp_forward.argtypes = [p, p, i32, p, p]
    L.mc_mlp_loss_grad.argtypes = [p, p, p, p, i32, p, p, p, p]
    L.mc_mlp_train.argtypes = [p, p, p, p, i32, i32, ctypes.c_float, p, ctypes.POINTER(i32), p, p, p]
    L.mc_mlp_targets.argtypes = [p, i32, i32, p, p, p]
    L.mc_mlp_predict_weights.argtypes = [p, i32, i32, p, p]
    for f in EXPORTED:
        if f not in ("mc_n_bins", "mc_trace_elem_bytes", "mc_lattice_words", "mc_last_error", "mc_mlp_n_params",
                     "mc_mlp_workspace_bytes"):
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(st):
    if st != MC_OK:
        raise MCError(st, lib().mc_last_error().decode())


def _dev_ptr(t, dtype, numel=None, name="tensor"):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, has %d" % (name, numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Chains of one or more lattice sizes on the current GPU (mc_create).

    sizes: list of (L, n_chains, seed, bin_shift) or (L, n_chains, seed,
    bin_shift, chain_offset) tuples.
    """

    def __init__(self, sizes, stream=None):
        import torch

        self.sizes = [tuple(s) for s in sizes]
        arr = (_Size * len(sizes))(*[_Size(int(s[0]), int(s[1]), int(s[2]), int(s[3]), int(s[4]) if len(s) > 4 else 0)
                                     for s in self.sizes])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().mc_create(arr, len(sizes), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().mc_destroy(self._h))  # refuses while graphs of the context exist
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- geometry ---------------------------------------------------------
    def n_bins(self, i=0):
        return lib().mc_n_bins(self._h, i)

    def trace_dtype(self, i=0):
        import torch

        return torch.int16 if lib().mc_trace_elem_bytes(self._h, i) == 2 else torch.int32

    def lattice_words(self, i=0):
        return lib().mc_lattice_words(self._h, i)

    def new_trace(self, n_sweeps, i=0):
        import torch

        return torch.empty((self.sizes[i][1], n_sweeps), dtype=self.trace_dtype(i), device="cuda")

    def new_hist(self, i=0):
        import torch

        return torch.zeros(self.n_bins(i), dtype=torch.int32, device="cuda")

    def new_cut(self, i=0):
        import torch

        return torch.empty(self.sizes[i][1], dtype=torch.int32, device="cuda")

    # -- the method -------------------------------------------------------
    def init_weights(self, lnW=None, i=0):
        nb = self.n_bins(i)
        if lnW is None:
            _check(lib().mc_init_weights(self._h, i, None, nb))
            return
        w = np.ascontiguousarray(np.asarray(lnW, dtype=np.float64))
        if w.size != nb:
            raise ValueError("lnW must have %d bins" % nb)
        _check(lib().mc_init_weights(self._h, i, w.ctypes.data_as(ctypes.c_void_p), nb))

    def run_chains(self, n_sweeps, traces, hists):
        """traces/hists: one tensor per size (or a single tensor for one size)."""
        import torch

        if isinstance(traces, torch.Tensor):
            traces = [traces]
        if isinstance(hists, torch.Tensor):
            hists = [hists]
        if len(traces) != len(self.sizes) or len(hists) != len(self.sizes):
            raise ValueError("need one trace and one hist per size")
        tp = (ctypes.c_void_p * len(self.sizes))()
        hp = (ctypes.c_void_p * len(self.sizes))()
        for i in range(len(self.sizes)):
            tp[i] = _dev_ptr(traces[i], self.trace_dtype(i), self.sizes[i][1] * n_sweeps, "trace").value
            hp[i] = _dev_ptr(hists[i], torch.int32, self.n_bins(i), "hist").value
        _check(lib().mc_run_chains(self._h, int(n_sweeps), tp, hp))

    def run_chains_part(self, n_sweeps, col, traces, hists):
        """Sweeps n_sweeps more of a round whose traces (one [n_chains][row_len]
        tensor per size) are filled from column col (mc_run_chains_part)."""
        import torch

        if isinstance(traces, torch.Tensor):
            traces = [traces]
        if isinstance(hists, torch.Tensor):
            hists = [hists]
        if len(traces) != len(self.sizes) or len(hists) != len(self.sizes):
            raise ValueError("need one trace and one hist per size")
        row_len = traces[0].shape[-1]
        tp = (ctypes.c_void_p * len(self.sizes))()
        hp = (ctypes.c_void_p * len(self.sizes))()
        for i in range(len(self.sizes)):
            if traces[i].shape[-1] != row_len:
                raise ValueError("every size's trace must have the same row length")
            tp[i] = _dev_ptr(traces[i], self.trace_dtype(i), self.sizes[i][1] * row_len, "trace").value
            hp[i] = _dev_ptr(hists[i], torch.int32, self.n_bins(i), "hist").value
        _check(lib().mc_run_chains_part(self._h, int(n_sweeps), int(col), int(row_len), tp, hp))

    def join(self, trace, cut, hist, mode=0, i=0):
        import torch

        M = trace.shape[-1]
        _check(lib().mc_join(self._h, i, _dev_ptr(trace, self.trace_dtype(i), self.sizes[i][1] * M, "trace"), int(M),
                             _dev_ptr(cut, torch.int32, self.sizes[i][1], "cut"),
                             _dev_ptr(hist, torch.int32, self.n_bins(i), "hist"), int(mode)))

    def update_weights(self, hist, i=0, want=True):
        """Returns (lnW numpy array, flat flag, retained count) when want."""
        import torch

        hp = _dev_ptr(hist, torch.int32, self.n_bins(i), "hist")
        if not want:
            _check(lib().mc_update_weights(self._h, i, hp, None, None, None))
            return None
        w = np.zeros(self.n_bins(i), dtype=np.float64)
        flat = ctypes.c_int32()
        ret = ctypes.c_int64()
        _check(lib().mc_update_weights(self._h, i, hp, w.ctypes.data_as(ctypes.c_void_p), ctypes.byref(flat),
                                       ctypes.byref(ret)))
        return w, bool(flat.value), int(ret.value)

    def iterate_topup(self, m_total, m_max, trace, hist, cut, mode=0, max_rounds=1000):
        """One iteration with Algorithm step 6 (one-size contexts).  trace has
        room for n_chains * m_max entries.  Returns (rounds, sweeps per chain,
        configurations kept, flat flag)."""
        import torch

        P = self.sizes[0][1]
        rounds, sweeps, kept, flat = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib().mc_iterate_topup(self._h, int(m_total), int(m_max), int(max_rounds),
                                      _dev_ptr(trace, self.trace_dtype(0), P * int(m_max), "trace"),
                                      _dev_ptr(hist, torch.int32, self.n_bins(0), "hist"),
                                      _dev_ptr(cut, torch.int32, P, "cut"), int(mode), ctypes.byref(rounds),
                                      ctypes.byref(sweeps), ctypes.byref(kept), ctypes.byref(flat)))
        return rounds.value, sweeps.value, kept.value, bool(flat.value)

    def get_state(self):
        """Checkpoint of the whole context as bytes (mc_get_state)."""
        n = ctypes.c_size_t(0)
        _check(lib().mc_get_state(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().mc_get_state(self._h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def set_state(self, blob):
        """Resume from a checkpoint taken by get_state (mc_set_state)."""
        blob = bytes(blob)
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().mc_set_state(self._h, buf, len(blob)))

    # -- inspection -------------------------------------------------------
    def levels(self, i=0):
        out = np.zeros(self.sizes[i][1], dtype=np.int32)
        _check(lib().mc_get_levels(self._h, i, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def lattice(self, chain, i=0):
        n = self.lattice_words(i)
        out = np.zeros(n, dtype=np.uint32)
        _check(lib().mc_get_lattice(self._h, i, chain, out.ctypes.data_as(ctypes.c_void_p), n))
        return out

    def spins(self, chain, i=0):
        """Lattice of one chain as +-1 int8 in site order j = y*L + x."""
        L = self.sizes[i][0]
        W = (L + 31) // 32
        words = self.lattice(chain, i).reshape(L, W)
        x = np.arange(L)
        bits = (words[:, x // 32] >> (x % 32).astype(np.uint32)) & 1
        return (bits.astype(np.int8) * 2 - 1).reshape(-1)

    def stats(self, i=0):
        """mc_get_stats of size i as a dict."""
        st = Stats()
        _check(lib().mc_get_stats(self._h, i, ctypes.byref(st)))
        return st.as_dict()

    def check_levels(self, i=0):
        """Recount every chain's broken bonds against its level
        (mc_check_levels); raises MCError (MC_EINTERNAL) on a disagreement."""
        n = ctypes.c_int64()
        _check(lib().mc_check_levels(self._h, i, ctypes.byref(n)))
        return n.value

    def counters(self, i=0):
        seam = ctypes.c_int32()
        rnd = ctypes.c_uint32()
        sw = ctypes.c_uint32()
        _check(lib().mc_get_counters(self._h, i, ctypes.byref(seam), ctypes.byref(rnd), ctypes.byref(sw)))
        return seam.value, rnd.value, sw.value

    def set_seam(self, seam, i=0):
        """The seam the next joint of size i starts from (mc_set_seam)."""
        _check(lib().mc_set_seam(self._h, i, int(seam)))

    def weights(self, i=0):
        w = np.zeros(self.n_bins(i), dtype=np.float64)
        _check(lib().mc_get_weights(self._h, i, w.ctypes.data_as(ctypes.c_void_p), self.n_bins(i)))
        return w

    def thermo(self, betas, i=0):
        """E, C, F, S (totals) at the inverse temperatures `betas` from the
        current ln w (mc_thermo); four float64 arrays."""
        b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64).ravel())
        out = np.zeros(4 * b.size, dtype=np.float64)
        _check(lib().mc_thermo(self._h, i, b.ctypes.data_as(ctypes.c_void_p), int(b.size),
                               out.ctypes.data_as(ctypes.c_void_p)))
        out = out.reshape(4, b.size)
        return out[0], out[1], out[2], out[3]

    def progress(self, i=0):
        """(updates done, first flat update or 0, last update flat, kept before last update)"""
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        r = ctypes.c_int64()
        _check(lib().mc_get_progress(self._h, i, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(r)))
        return a.value, b.value, bool(c.value), r.value

    # -- launch configuration (speed only, never results) ------------------
    def set_chains_per_block(self, cpb, i=0):
        _check(lib().mc_set_chains_per_block(self._h, i, int(cpb)))

    def set_launch(self, kind, cpb, i=0):
        """Kernel kind and chains per workgroup of size i (mc_set_launch)."""
        _check(lib().mc_set_launch(self._h, i, int(kind), int(cpb)))

    def launch(self, i=0):
        """(chains per block, kernel kind, batched flag)"""
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().mc_get_launch(self._h, i, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, bool(c.value)

    def autotune(self, probe_sweeps=20):
        out = (ctypes.c_int32 * len(self.sizes))()
        _check(lib().mc_autotune(self._h, int(probe_sweeps), out))
        return list(out)

    def graph(self, n_sweeps, n_iters, traces, hists, cuts, mode=0):
        return Graph(self, n_sweeps, n_iters, traces, hists, cuts, mode)

    def sync(self):
        _check(lib().mc_sync(self._h))


class Graph:
    """n_iters captured iterations (run + join + update of every size)."""

    def __init__(self, ctx, n_sweeps, n_iters, traces, hists, cuts, mode=0):
        import torch

        n = len(ctx.sizes)
        if not (len(traces) == len(hists) == len(cuts) == n):
            raise ValueError("need one trace, hist and cut buffer per size")
        tp = (ctypes.c_void_p * n)()
        hp = (ctypes.c_void_p * n)()
        cp = (ctypes.c_void_p * n)()
        for i in range(n):
            tp[i] = _dev_ptr(traces[i], ctx.trace_dtype(i), ctx.sizes[i][1] * n_sweeps, "trace").value
            hp[i] = _dev_ptr(hists[i], torch.int32, ctx.n_bins(i), "hist").value
            cp[i] = _dev_ptr(cuts[i], torch.int32, ctx.sizes[i][1], "cut").value
        self._keep = (traces, hists, cuts)  # the graph reads and writes these buffers
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib().mc_graph_create(ctx._h, int(n_sweeps), int(n_iters), tp, hp, cp, int(mode), ctypes.byref(h)))
        self._h = h

    def launch(self):
        _check(lib().mc_graph_launch(self.ctx._h, self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().mc_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PROBES = {0: "valu_xor", 1: "valu_mul_lo", 2: "valu_mul_hi", 3: "valu_mad_u64", 4: "valu_bitop3",
          5: "lds_read_bandwidth", 6: "lds_dependent_read_cycles", 7: "lone_wave_dependent_issue_cycles",
          8: "lone_wave_independent_issue_cycles", 9: "quad_step_cycles", 10: "quad_step_cycles_pair_table_reads",
          11: "quad_step_cycles_no_threshold_reads"}


def probe(kind, iters, stream=None):
    """mc_probe: (figure, seconds, work, cycles) of one microbenchmark."""
    out = np.zeros(4, dtype=np.float64)
    _check(lib().mc_probe(int(kind), int(iters), _stream_ptr(stream), out.ctypes.data_as(ctypes.c_void_p)))
    return tuple(float(v) for v in out)


# --------------------------------------------------------------------------- #
# Learned initial weight (the 2-64-64-1 tanh network of mc.h)                 #
# --------------------------------------------------------------------------- #
def _stream_ptr(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def mlp_n_params():
    return int(lib().mc_mlp_n_params())


class MLP:
    """Parameters, Adam state and workspace of one network on the GPU."""

    def __init__(self, seed=1, params=None, stream=None):
        import torch

        self.n_params = mlp_n_params()
        self.stream = stream
        if params is None:
            self.params = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
            _check(lib().mc_mlp_init(_dev_ptr(self.params, torch.float32), int(seed), _stream_ptr(stream)))
        else:
            self.params = torch.as_tensor(params, dtype=torch.float32).cuda().contiguous()
        self.adam = torch.zeros(2 * self.n_params, dtype=torch.float32, device="cuda")
        self.step = ctypes.c_int32(0)
        self._ws = None

    def _workspace(self, n):
        import torch

        need = int(lib().mc_mlp_workspace_bytes(int(n)))
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        return ctypes.c_void_p(self._ws.data_ptr())

    def forward(self, x):
        import torch

        x = x.contiguous()
        n = x.numel() // 2
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        _check(lib().mc_mlp_forward(_dev_ptr(self.params, torch.float32), _dev_ptr(x, torch.float32), n,
                                    _dev_ptr(y, torch.float32), _stream_ptr(self.stream)))
        return y

    def loss_grad(self, x, t, w=None):
        import torch

        n = t.numel()
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().mc_mlp_loss_grad(_dev_ptr(self.params, torch.float32), _dev_ptr(x, torch.float32),
                                      _dev_ptr(t, torch.float32), _dev_ptr(w, torch.float32) if w is not None else None,
                                      n, _dev_ptr(g, torch.float32), _dev_ptr(loss, torch.float32),
                                      self._workspace(n), _stream_ptr(self.stream)))
        return loss, g

    def train(self, x, t, w=None, steps=1000, lr=1e-3):
        """Full-batch Adam steps; returns the loss before the last step."""
        import torch

        n = t.numel()
        loss = ctypes.c_float()
        _check(lib().mc_mlp_train(_dev_ptr(self.params, torch.float32), _dev_ptr(x, torch.float32),
                                  _dev_ptr(t, torch.float32), _dev_ptr(w, torch.float32) if w is not None else None,
                                  n, int(steps), float(lr), _dev_ptr(self.adam, torch.float32), ctypes.byref(self.step),
                                  ctypes.byref(loss), self._workspace(n), _stream_ptr(self.stream)))
        return float(loss.value)

    def predict_weights(self, L, bin_shift=1):
        """Proposed ln w (numpy, fp64) of an L x L lattice."""
        import torch

        nb = ((L * L) >> bin_shift) + 1
        w = torch.empty(nb, dtype=torch.float64, device="cuda")
        _check(lib().mc_mlp_predict_weights(_dev_ptr(self.params, torch.float32), int(L), int(bin_shift),
                                            _dev_ptr(w, torch.float64), _stream_ptr(self.stream)))
        return w.cpu().numpy()


def mlp_targets(lnW, L, bin_shift=1, stream=None):
    """Training samples (x [n][2], t [n]) of a converged ln w, built on the GPU."""
    import torch

    w = torch.as_tensor(np.asarray(lnW, dtype=np.float64)).cuda().contiguous()
    nb = w.numel()
    x = torch.empty((nb, 2), dtype=torch.float32, device="cuda")
    t = torch.empty(nb, dtype=torch.float32, device="cuda")
    _check(lib().mc_mlp_targets(_dev_ptr(w, torch.float64), int(L), int(bin_shift), _dev_ptr(x, torch.float32),
                                _dev_ptr(t, torch.float32), _stream_ptr(stream)))
    return x, t
