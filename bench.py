"""Benchmark: parallel multicanonical Metropolis chains on the 2D Ising model
(arXiv 0812.2964, Algorithm steps 2-5 and eq. new_weight) on one MI355X.

Workload (default): L = 32, 4096 chains x 10^5 sweeps per step, width-8 energy
bins (513), the prior ln w of tests/golden/lnW_L32_prior.npy, seed 1.
One step = mc_run_chains (10^5 sweeps of every chain) + mc_join (detailed-balance
joints over all 4096 chains) + mc_update_weights (eq. new_weight + flatness +
re-tabulation).  Inputs are resident in device memory before timing starts.

Prints one JSON line (rank 0) with the throughput in spin-flip attempts/s, the
sweep kernel's position against the integer-ALU roofline, and the CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Integer operations one Metropolis attempt needs, counted from the method:
#   Philox4x32-10, one call per 4 words: 10 rounds x (2 mulhi + 2 mullo + 4 xor) = 80 -> 20 / attempt
#   neighbour count (4 xor + 3 add), threshold index (1), compare (1), flip (1), level update (1) = 11
OPS_PER_ATTEMPT = 31
# MI355X: 256 CUs x 64 lanes x 2.4 GHz of full-rate 32-bit vector ALU operations.
ALU_PEAK_OPS = 256 * 64 * 2.4e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=32)
    ap.add_argument("--chains", type=int, default=4096)
    ap.add_argument("--sweeps", type=int, default=100000)
    ap.add_argument("--cpu-chains", type=int, default=64)
    ap.add_argument("--cpu-sweeps", type=int, default=4000)
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def traffic_from_profiles(L, P, M):
    """HBM bytes per sweep launch from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "sweep_L32_4096x1e5_counters.md")
    src = os.path.join(ROOT, "paper_0812_2964_amd", "csrc", "mc_kernels.hip")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel source sha256:\s*([0-9a-f]{64})", txt)
    m_bytes = re.search(r"HBM bytes per launch \(scaled\):\s*([0-9.eE+]+)", txt)
    m_cfg = re.search(r"workload:\s*L=(\d+) chains=(\d+) sweeps=(\d+)", txt)
    if not (m_hash and m_bytes and m_cfg):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_hash.group(1):
        return None
    if (int(m_cfg.group(1)), int(m_cfg.group(2)), int(m_cfg.group(3))) != (L, P, M):
        return None
    return float(m_bytes.group(1))


def cpu_baseline(L, lnW, chains, sweeps):
    import oracle as O

    R = O.Run(L, chains, seed=1, bin_shift=1, lnW=lnW)
    t0 = time.perf_counter()
    R.run(sweeps, want_trace=True)
    dt = time.perf_counter() - t0
    att = chains * sweeps * L * L
    return {"value": att / dt, "unit": "spin-flip attempts/s", "cores": 1, "kind": "oracle",
            "sample": "%d chains x %d sweeps of the same L=%d workload (%.3g attempts, %.1f s, single thread)"
                      % (chains, sweeps, L, att, dt)}


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the method's chains live on a single device here "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_0812_2964_amd as mc

    torch.cuda.set_device(0)
    L, P, M = a.L, a.chains, a.sweeps
    N = L * L
    lnW = np.load(os.path.join(ROOT, "tests", "golden", "lnW_L32_prior.npy")) if L == 32 else None
    stream = torch.cuda.current_stream()
    ctx = mc.Context([(L, P, 1, 1)], stream=stream)
    ctx.init_weights(lnW)
    trace = ctx.new_trace(M)
    hist = ctx.new_hist()
    cut = ctx.new_cut()
    log("bench: L=%d chains=%d sweeps=%d, warmup %d, steps %d" % (L, P, M, a.warmup, a.steps))

    ev = []

    def step(timed):
        if timed:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        ctx.run_chains(M, trace, hist)
        if timed:
            e1.record(stream)
            ev.append((e0, e1))
        ctx.join(trace, cut, hist)
        ctx.update_weights(hist, want=False)

    for w in range(a.warmup):
        step(False)
        torch.cuda.synchronize()
        log("bench: warmup step %d done" % (w + 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        step(True)
        torch.cuda.synchronize()
        log("bench: step %d done (%.2f s so far)" % (s + 1, time.perf_counter() - t0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sweep_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    attempts_step = P * M * N
    value = a.steps * attempts_step / elapsed
    avg_sweep_s = sum(sweep_ms) / len(sweep_ms) / 1e3
    achieved = attempts_step * OPS_PER_ATTEMPT / avg_sweep_s
    seam, rnd, sweep_idx = ctx.counters()
    res = {
        "metric": "spin-flip attempts/s (multicanonical Ising, 1 GPU); iterations to flat H",
        "value": value,
        "unit": "spin-flip attempts/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "2D Ising L=%d periodic, %d chains x %d sweeps per step (run + joint + weight "
                               "update), width-8 energy bins, prior ln w fixture, seed 1" % (L, P, M),
                   "L": L, "chains": P, "sweeps_per_step": M, "bins": ctx.n_bins(), "parallelism": "chains"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_OPS / 1e12, "unit": "Tops/s",
                     "frac": achieved / ALU_PEAK_OPS, "traffic": traffic_from_profiles(L, P, M),
                     "kernel": "k_sweep (mc_run_chains)", "kernel_ms": avg_sweep_s * 1e3,
                     "ops_per_attempt": OPS_PER_ATTEMPT},
        "sweep_attempts_per_s": attempts_step / avg_sweep_s,
    }
    ctx.close()
    if not a.no_cpu:
        log("bench: timing the CPU oracle on a sample")
        res["cpu_baseline"] = cpu_baseline(L, lnW, a.cpu_chains, a.cpu_sweeps)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
