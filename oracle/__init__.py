"""ctypes front end of the CPU oracle (test infrastructure only).

The oracle is the plain, serial, fp64 statement of what the GPU path computes
(parallel multicanonical Metropolis chains, the detailed-balance joint and the
weight recursion of arXiv 0812.2964).  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import this package; the product
path never does.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_u32 = ctypes.c_uint32
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_p = ctypes.c_void_p


def lib():
    """Load liboracle.so, building it with gcc first if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path):
        _build.build()
    L = ctypes.CDLL(path)
    L.orc_philox4x32_10.argtypes = [_p, _p, _p]
    L.orc_uniform.argtypes = [_u32, _i32, _u32, _u32, _u32, _u32]
    L.orc_uniform.restype = _u32
    L.orc_exp.argtypes = [_dbl]
    L.orc_exp.restype = _dbl
    L.orc_log.argtypes = [_i64]
    L.orc_log.restype = _dbl
    L.orc_threshold.argtypes = [_dbl]
    L.orc_threshold.restype = _u32
    L.orc_energy.argtypes = [_i32, _p]
    L.orc_energy.restype = _i64
    L.orc_init_chain.argtypes = [_i32, _u32, _u32, _p]
    L.orc_level_reachable.argtypes = [_i32, _i32]
    L.orc_level_reachable.restype = ctypes.c_int
    L.orc_tabulate.argtypes = [_i32, _i32, _p, _p]
    L.orc_sweeps.argtypes = [_i32, _u32, _i32, _u32, _p, _p, _u32, _i64, _p, _p, _p]
    L.orc_join.argtypes = [_i32, _i32, _u32, _u32, _i32, _i64, _p, _p, _p, _u32, _i32, _p, _p, _p, _p]
    L.orc_energy_order.argtypes = [_i32, _p, _p, _i32, _p]
    L.orc_update.argtypes = [_i32, _i32, _p, _p]
    L.orc_update.restype = ctypes.c_int
    L.orc_run_round.argtypes = [_i32, _u32, _i32, _u32, _i32, _i64, _u32, _p, _p, _p, _p, _p]
    if hasattr(L, "orc_mlp_forward"):
        _bind_mlp(L)
    _lib = L
    return L


def _bind_mlp(L):
    L.orc_mlp_n_params.restype = _i32
    L.orc_mlp_forward.argtypes = [_p, _p, _i32, _p]
    L.orc_mlp_loss_grad.argtypes = [_p, _p, _p, _p, _i32, _p]
    L.orc_mlp_loss_grad.restype = _dbl


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------- #
# Elementary pieces                                                           #
# --------------------------------------------------------------------------- #
def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed, L, dom, a, c, j):
    return int(lib().orc_uniform(seed, L, dom, a, c, j))


def det_exp(x):
    return float(lib().orc_exp(float(x)))


def det_log(h):
    return float(lib().orc_log(int(h)))


def threshold(d):
    return int(lib().orc_threshold(float(d)))


def mlp_n_params():
    return int(lib().orc_mlp_n_params())


def mlp_forward(params, x):
    """fp64 forward of the 2-64-64-1 tanh network; x: (n, 2)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    y = np.zeros(len(xx))
    lib().orc_mlp_forward(_ptr(p), _ptr(xx), len(xx), _ptr(y))
    return y


def mlp_loss_grad(params, x, t, w=None):
    """Weighted mean squared error and its gradient (fp64)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    tt = np.ascontiguousarray(t, dtype=np.float64)
    ww = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    g = np.zeros(mlp_n_params())
    loss = lib().orc_mlp_loss_grad(_ptr(p), _ptr(xx), _ptr(tt), _ptr(ww) if ww is not None else None, len(xx),
                                   _ptr(g))
    return float(loss), g


def n_bins(L, bin_shift):
    return ((L * L) >> bin_shift) + 1


def energy(L, spins):
    s = np.ascontiguousarray(spins, dtype=np.int8)
    assert s.size == L * L
    return int(lib().orc_energy(L, _ptr(s)))


def init_chain(L, seed, c):
    s = np.zeros(L * L, dtype=np.int8)
    lib().orc_init_chain(L, seed, c, _ptr(s))
    return s


def level_reachable(L, m):
    return bool(lib().orc_level_reachable(L, m))


def reachable_bins(L, bin_shift):
    N = L * L
    nb = n_bins(L, bin_shift)
    r = np.zeros(nb, dtype=bool)
    for m in range(N + 1):
        if level_reachable(L, m):
            r[m >> bin_shift] = True
    return r


def tabulate(L, bin_shift, lnW):
    lnW = np.ascontiguousarray(lnW, dtype=np.float64)
    assert lnW.size == n_bins(L, bin_shift)
    T = np.zeros((L * L + 1) * 5, dtype=np.uint32)
    lib().orc_tabulate(L, bin_shift, _ptr(lnW), _ptr(T))
    return T.reshape(L * L + 1, 5)


def sweeps(L, seed, bin_shift, c, spins, m, g0, M, lnW):
    """Run M sweeps of chain c from (spins, m); returns (spins, m, trace, hist)."""
    T = np.ascontiguousarray(tabulate(L, bin_shift, lnW).ravel())
    s = np.ascontiguousarray(spins, dtype=np.int8).copy()
    mm = np.array([m], dtype=np.int32)
    tr = np.zeros(M, dtype=np.int32)
    h = np.zeros(n_bins(L, bin_shift), dtype=np.int64)
    lib().orc_sweeps(L, seed, bin_shift, c, _ptr(s), _ptr(mm), g0, M, _ptr(T), _ptr(tr), _ptr(h))
    return s, int(mm[0]), tr, h


def energy_order(first, last, sigma):
    """The energy ordering of the chains for one round (greedy chain of
    nearest levels from the seam; see orc_energy_order).  first, last: levels
    of each chain's first and last configuration."""
    first = np.ascontiguousarray(first, dtype=np.int32)
    last = np.ascontiguousarray(last, dtype=np.int32)
    order = np.zeros(first.size, dtype=np.int32)
    lib().orc_energy_order(first.size, _ptr(first), _ptr(last), sigma, _ptr(order))
    return order


def join(L, bin_shift, seed, trace, lnW, sigma, r, mode=0, chain_offset=0):
    """Join one round.  trace: (p, M) array of E/4.  mode 0: detailed balance
    in chain order; 1: naive splice; 2: detailed balance with the chains in
    energy order.  chain_offset: global index of the first chain (a block of a
    split run).  Returns (cut, H, retained, new_sigma)."""
    tr = np.ascontiguousarray(trace, dtype=np.int32)
    p, M = tr.shape
    lnW = np.ascontiguousarray(lnW, dtype=np.float64)
    sig = np.array([sigma], dtype=np.int32)
    cut = np.zeros(p, dtype=np.int32)
    H = np.zeros(n_bins(L, bin_shift), dtype=np.int64)
    ret = np.zeros(1, dtype=np.int64)
    order = None
    if mode == 2:
        half = L * L // 2
        order = energy_order(tr[:, 0] + half, tr[:, M - 1] + half, sigma)
    lib().orc_join(L, bin_shift, seed, chain_offset, p, M, _ptr(tr), _ptr(lnW), _ptr(sig), r, 1 if mode == 1 else 0,
                   _ptr(order) if order is not None else None, _ptr(cut), _ptr(H), _ptr(ret))
    return cut, H, int(ret[0]), int(sig[0])


def topup_sweeps(m_total, m_max, kept, swept):
    """Sweeps of the next round of Algorithm step 6: the shortfall
    m_total - kept at the rate kept / swept seen so far (kept configurations
    per sweep of all chains), rounded up, within 1 .. m_max; m_max while
    nothing has been kept.  Integers only."""
    if kept <= 0:
        return m_max
    need = m_total - kept
    return max(1, min(m_max, -(-need * swept // kept)))


def update(L, bin_shift, H, lnW):
    """Eq. (new_weight) in logs.  Returns (new lnW, flat flag)."""
    H = np.ascontiguousarray(H, dtype=np.int64)
    w = np.ascontiguousarray(lnW, dtype=np.float64).copy()
    flat = lib().orc_update(L, bin_shift, _ptr(H), _ptr(w))
    return w, bool(flat)


# --------------------------------------------------------------------------- #
# A whole run: p chains of one lattice size, the state carried across rounds  #
# and weight updates as the paper's Sec. 2 remarks prescribe.                 #
# --------------------------------------------------------------------------- #
class Run:
    def __init__(self, L, n_chains, seed=1, bin_shift=1, lnW=None, chain_offset=0):
        self.L, self.p, self.seed, self.bin_shift = L, n_chains, seed, bin_shift
        self.N = L * L
        self.nb = n_bins(L, bin_shift)
        self.c0 = chain_offset
        self.spins = np.stack([init_chain(L, seed, chain_offset + c) for c in range(n_chains)]).astype(np.int8)
        self.m = np.array([(energy(L, s) + 2 * self.N) // 4 for s in self.spins], dtype=np.int32)
        self.lnW = np.zeros(self.nb) if lnW is None else np.array(lnW, dtype=np.float64)
        self.g = 0          # global sweep index
        self.r = 0          # round index of the joint
        self.sigma = -1     # seam level, -1 = none
        self.H = np.zeros(self.nb, dtype=np.int64)
        self.retained = 0

    def run(self, M, want_trace=True):
        """Algorithm step 2 for all chains.  Returns (trace (p, M) of E/4,
        raw histogram over all chains)."""
        tr = np.zeros((self.p, M), dtype=np.int32) if want_trace else None
        hist = np.zeros(self.nb, dtype=np.int64)
        spins = np.ascontiguousarray(self.spins)
        lnW = np.ascontiguousarray(self.lnW)
        lib().orc_run_round(self.L, self.seed, self.bin_shift, self.c0, self.p, M, self.g, _ptr(lnW), _ptr(spins),
                            _ptr(self.m), _ptr(tr) if tr is not None else None, _ptr(hist))
        self.spins = spins
        self.g += M
        return tr, hist

    def join(self, trace, mode=0):
        cut, H, ret, self.sigma = join(self.L, self.bin_shift, self.seed, trace, self.lnW, self.sigma, self.r, mode,
                                       self.c0)
        self.r += 1
        self.H += H
        self.retained += ret
        return cut, H

    def update(self):
        self.lnW, flat = update(self.L, self.bin_shift, self.H, self.lnW)
        self.H[:] = 0
        self.retained = 0
        return flat

    def iterate_topup(self, m_total, m_max, mode=0):
        """One iteration with Algorithm step 6: rounds of m sweeps and joints
        until the joined histogram holds at least m_total configurations,
        then the weight update.  Returns (sweeps of each round, retained,
        flat, traces of each round)."""
        rounds, traces = [], []
        kept0 = self.retained
        swept = 0
        while True:
            m = topup_sweeps(m_total, m_max, self.retained - kept0, swept) if rounds else m_max
            tr, _ = self.run(m)
            self.join(tr, mode)
            rounds.append(m)
            traces.append(tr)
            swept += m
            if self.retained - kept0 >= m_total:
                break
        retained = self.retained
        flat = self.update()
        return rounds, retained, flat, traces
