"""Benchmark: parallel multicanonical Metropolis chains on the 2D Ising model
(arXiv 0812.2964: Algorithm steps 2-5 and eq. new_weight) on one MI355X.

Default workload (the one the headline metric is quoted on): lattices of
uneven size L in {16, 24, 32, 48, 64}, 2048 chains each, in one persistent
launch; 10^5 sweeps per iteration, width-8 energy bins, ln w = 0 at the
start, seed 1.  One step = one iteration of the recursion for all five sizes,
replayed from a HIP graph: the sweeps of every chain (Algorithm step 2), the
detailed-balance joints over each size's chains (steps 3-5) and the weight
updates (eq. new_weight, flatness, re-tabulation).  The warmup steps are the
recursion's first iterations, the timed steps the following ones; iterations
to the first flat histogram are reported per size.  Inputs and state are
resident in device memory before the timed region.

Prints one JSON line with the throughput in spin-flip attempts/s, the sweep
kernel against the integer-ALU roofline (and against the ceiling set by one
wave's issue rate for serial chains), and the CPU oracle timed on a bounded
sample of the same workload.

Other workloads (--workload): l32 (L = 32, 4096 chains x 10^5 sweeps, the
prior ln w fixture), recursion8 (L = 8, 16 chains, 10^4 sweeps, ten
iterations from ln w = 0), large (L = 128, 8192 chains x 2 x 10^5 sweeps per
iteration from ln w = 0, checkpointed across calls; --lattice 100 or 256),
l128 (short runs of the large lattices for profiling), thermo (the reduced
reweighting of code (ii) at L = 256 for 4096 inverse temperatures), fig2 (the
comparison of Fig. 2: detailed-balance joints against naive splices at L = 20,
measured by code (ii) against the exact energy), fig1 (the comparison of
Fig. 1 at L = 64 and the paper's L = 100: weights from the learned
initialiser, E, C, F, S of code (ii) against the exact finite lattice), topup
(Algorithm step 6 with joints in chain order, in energy order and naive, at
L = 20), learned (iterations to flat at L = 64 from the network's proposal
against ln w = 0), learned256 (the network trained on converged weights of
smaller lattices initialises L = 256, 4096 chains, against ln w = 0), peaks
(the microbenchmarks of mc_probe) and copy (a plain device copy of known size,
to calibrate the HBM byte counters).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Integer operations one Metropolis attempt needs, counted from the method as
# two-operand operations (independent of any instruction set's fused forms):
#   Philox4x32-10, one call per 4 words: 10 rounds x (2 mulhi + 2 mullo + 4 xor) = 80 -> 20 / attempt
#   neighbour count (4 xor + 3 add), threshold index (1), compare (1), flip (1), level update (1) = 11
OPS_PER_ATTEMPT = 31
# MI355X: 256 CUs x 128 lanes x 2.4 GHz of 32-bit vector ALU operations per
# second (the published fp32 vector peak, 157.3 TFLOP/s, is 128 fused
# multiply-adds per clock per CU; mc_probe measures 73-85 % of this figure for
# v_xor_b32 and v_bitop3_b32 alone, so simple 32-bit integer operations run at
# that width too, and 32-bit multiplies at about half of it).
CLOCK_HZ = 2.4e9
ALU_LANES_PER_CLK_PER_CU = 128
ALU_PEAK_OPS = 256 * ALU_LANES_PER_CLK_PER_CU * CLOCK_HZ
METRIC = "spin-flip attempts/s (multicanonical Ising, 1 GPU); iterations to flat H"
BATCHED_LS = [16, 24, 32, 48, 64]
# VALU instructions the consumer wave of a chain issues per step of four sites,
# counted in the compiled code of the step (the instructions between two
# selections of the quad's result in the unrolled row loop): the quad kernel
# (kind 7, in the batched launch at L = 64 and alone at L = 32) and the
# large-lattice quad kernel in the parity state (kinds 8, 9 at L = 128).  A chain's attempts are
# serial and its wave issues one VALU instruction per issue interval at best,
# so 4 sites take at least valu_per_step x interval cycles.
CONSUMER_VALU_PER_STEP = {7: 37, 8: 60, 9: 60}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched",
                    choices=["batched", "l32", "recursion8", "large", "l128", "thermo", "fig1", "fig2", "topup",
                             "learned", "learned256", "peaks", "copy"])
    ap.add_argument("--rounds", type=int, default=None)
    ap.add_argument("--chains", type=int, default=None)
    ap.add_argument("--sweeps", type=int, default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--lattice", type=int, default=128, help="l128: the lattice size (100, 128 or 256)")
    ap.add_argument("--cpu-chains", type=int, default=64)
    ap.add_argument("--cpu-sweeps", type=int, default=4000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--out-npz", default=None, help="fig1: also save the L = 64 and L = 100 weights there")
    ap.add_argument("--metrics", default=None, help="write one JSON line of recursion statistics per iteration and "
                                                      "size to this file")
    ap.add_argument("--state-in", default=None, help="large: resume from this checkpoint")
    ap.add_argument("--state-out", default=None, help="large: checkpoint to this file after every iteration")
    ap.add_argument("--parts", type=int, default=4, help="large: launches per round (progress between them)")
    ap.add_argument("--stage128", type=int, default=0, help="learned256: also run L = 128 from the network's "
                    "proposal for at most this many iterations, and train on it if it flattens")
    ap.add_argument("--no-arms", action="store_true", help="learned256: stop after the training stages")
    ap.add_argument("--graph-iters", type=int, default=1, help="batched: iterations captured in each timed graph "
                    "(--steps a multiple of it; the warmup then runs as one graph of --warmup iterations)")
    ap.add_argument("--budget-s", type=float, default=None, help="large: start no iteration that would end after "
                                                                  "this many seconds since the start")
    return ap.parse_args()


def kernel_source_hash():
    """sha256 over the sources the sweep kernel is compiled from."""
    h = hashlib.sha256()
    for f in ("mc_kernels.hip", "mc_math.h", "mc_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_0812_2964_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic_from_profiles(name, workload):
    """HBM bytes per sweep launch from the committed counter summary
    profiles/<name>, if it was taken on the current kernel source and the
    same workload (its "workload:" line); else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel source sha256:\s*([0-9a-f]{64})", txt)
    m_bytes = re.search(r"HBM bytes per launch \(scaled\):\s*([0-9.eE+]+)", txt)
    m_cfg = re.search(r"workload:[ \t]*([^\n]+)", txt)
    if not (m_hash and m_bytes and m_cfg):
        return None
    if kernel_source_hash() != m_hash.group(1) or m_cfg.group(1).strip() != workload:
        return None
    return float(m_bytes.group(1))


def issue_interval(mc):
    """A lone wave's issue interval for independent VALU instructions
    (mc_probe kind 8), in shader-clock cycles, and the shader clock the probe
    saw (its cycles over its event time)."""
    cyc, sec, _, cycles = mc.probe(8, 1 << 14)
    return cyc, cycles / sec


def chain_ceiling(mc, kind, attempts_per_launch, serial_attempts):
    """The ceiling serial chains put on one launch: the chain with the most
    attempts (serial_attempts = sweeps x sites of the largest lattice, run by
    kernel kind `kind`) cannot finish before its consumer wave has issued
    valu_per_step VALU instructions per four sites, one per issue interval at
    best.  None for kinds whose step is not counted."""
    if kind not in CONSUMER_VALU_PER_STEP:
        return None
    t, f = issue_interval(mc)
    cycles_per_attempt = CONSUMER_VALU_PER_STEP[kind] * t / 4.0
    launch_s = serial_attempts * cycles_per_attempt / CLOCK_HZ
    return {"attempts_per_s": attempts_per_launch / launch_s, "valu_per_step": CONSUMER_VALU_PER_STEP[kind],
            "sites_per_step": 4, "issue_cycles": t, "probe_clock_hz": f,
            "cycles_per_attempt_floor": cycles_per_attempt, "kernel_kind": kind}


def iteration_record(ctx, i, L, P, M, step, ms):
    """One line of recursion statistics (mc_get_stats) for size i after an
    iteration: retention, joints that kept nothing, cut points, flatness
    ratio min h / mean h over the reachable bins, ln w span, step time."""
    st = ctx.stats(i)
    kept_chains = P - st["join_none"]
    return {"L": L, "iteration": st["updates"], "step": step, "chains": P, "sweeps": M,
            "retained_frac": st["retained_last"] / float(P * M), "n_no_accept": st["join_none"],
            "mean_cut": st["join_cut_sum"] / kept_chains if kept_chains else None, "max_cut": st["join_cut_max"],
            "flat_ratio": st["hist_min"] * st["n_reach_bins"] / float(st["hist_sum"]) if st["hist_sum"] else 0.0,
            "flat": bool(st["last_flat"]), "first_flat": st["first_flat"] or None,
            "lnW_span": st["lnw_max"] - st["lnw_min"], "step_ms": ms}


class Metrics:
    """Per-iteration JSON lines (--metrics), or nothing."""

    def __init__(self, path):
        self.f = open(path, "a") if path else None

    def write(self, rec):
        if self.f:
            self.f.write(json.dumps(rec) + "\n")
            self.f.flush()

    def close(self):
        if self.f:
            self.f.close()


def cpu_threads():
    """Host threads for the oracle: the cores this process may run on, at most
    16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(L, lnW, chains, sweeps):
    """The oracle on the host: one thread over `chains` chains, then every
    usable core, each thread running its own contiguous block of chains/4
    chains (chains are independent; each block keys its random words by the
    global chain index, as a split run does), so that both legs together stay
    near 20 core-seconds.  The value is the all-core rate; the single-thread
    rate is kept beside it."""
    import threading

    import oracle as O

    R = O.Run(L, chains, seed=1, bin_shift=1, lnW=lnW)
    t0 = time.perf_counter()
    R.run(sweeps, want_trace=True)
    dt1 = time.perf_counter() - t0
    att1 = chains * sweeps * L * L
    T = cpu_threads()
    blk = max(1, chains // 4)
    runs = [O.Run(L, blk, seed=1, bin_shift=1, lnW=lnW, chain_offset=t * blk) for t in range(T)]
    threads = [threading.Thread(target=r.run, args=(sweeps, True)) for r in runs]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    dtT = time.perf_counter() - t0
    attT = T * blk * sweeps * L * L
    return {"value": attT / dtT, "unit": "spin-flip attempts/s", "cores": T, "kind": "oracle",
            "single_thread_value": att1 / dt1,
            "sample": "%d threads x %d chains x %d sweeps of the same L=%d workload (%.3g attempts, %.1f s); "
                      "single thread: %d chains x %d sweeps (%.1f s)"
                      % (T, blk, sweeps, L, attT, dtT, chains, sweeps, dt1)}


def base_record(a, value, ms_per_step, config, dtype="u32"):
    return {"metric": METRIC, "value": value, "unit": "spin-flip attempts/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def kernel_name(kind, L):
    return {0: "k_sweep_lds<%d,true>", 1: "k_sweep_lds<%d,false>", 2: "k_sweep_glb<%d>", 3: "k_sweep_generic",
            4: "k_sweep_pc<%d>", 5: "k_sweep_big<%d,true>", 6: "k_sweep_big<%d,false>",
            7: "k_sweep_pcq<%d>", 8: "k_sweep_bigq<%d,true>", 9: "k_sweep_bigq<%d,false>"}[kind].replace("%d", str(L))


def roofline(attempts, kernel_s, traffic):
    achieved = attempts * OPS_PER_ATTEMPT / kernel_s
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_OPS / 1e12, "unit": "Tops/s",
            "frac": achieved / ALU_PEAK_OPS, "traffic": traffic, "ops_per_attempt": OPS_PER_ATTEMPT,
            "kernel_ms": kernel_s * 1e3}


def bench_l32(a, torch, mc):
    L = 32
    P = a.chains or 4096
    M = a.sweeps or 100000
    N = L * L
    lnW = np.load(os.path.join(ROOT, "tests", "golden", "lnW_L32_prior.npy"))
    stream = torch.cuda.current_stream()
    ctx = mc.Context([(L, P, 1, 1)], stream=stream)
    ctx.init_weights(lnW)
    trace, hist, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
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
        # the workload samples at the fixed prior weight: restore it after
        # the update (which also clears the histogram for the next step)
        ctx.init_weights(lnW)

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
    sweep_s = sum(e0.elapsed_time(e1) for e0, e1 in ev) / len(ev) / 1e3
    att = P * M * N
    cpb, kind, _ = ctx.launch()
    res = base_record(a, a.steps * att / elapsed, elapsed / a.steps * 1e3,
                      {"workload": "2D Ising L=%d periodic, %d chains x %d sweeps per step (run + joint + weight "
                                   "update), width-8 energy bins, prior ln w fixture, seed 1" % (L, P, M),
                       "L": L, "chains": P, "sweeps_per_step": M, "bins": ctx.n_bins(), "parallelism": "chains",
                       "chains_per_block": cpb, "kernel_kind": kind})
    res["roofline"] = roofline(att, sweep_s, traffic_from_profiles("k_sweep_pcq_L32_4096x1e5_counters.md",
                                                                   "L=%d chains=%d sweeps=%d" % (L, P, M)))
    res["roofline"]["kernel"] = kernel_name(kind, L) + " (mc_run_chains)"
    res["sweep_attempts_per_s"] = att / sweep_s
    ctx.close()
    if not a.no_cpu:
        log("bench: timing the CPU oracle on a sample")
        res["cpu_baseline"] = cpu_baseline(L, lnW, a.cpu_chains, a.cpu_sweeps)
    return res


def bench_recursion8(a, torch, mc):
    """L = 8, 16 chains, 10^4 sweeps, ten iterations of the recursion from ln w = 0."""
    L, P = 8, a.chains or 16
    M = a.sweeps or 10000
    iters = a.iters or 10
    ctx = mc.Context([(L, P, 1, 1)])
    trace, hist, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
    g = ctx.graph(M, iters, [trace], [hist], [cut])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.launch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    upd, first_flat, last_flat, _ = ctx.progress()
    g.close()
    ctx.close()
    res = base_record(a, iters * P * M * L * L / dt, dt * 1e3,
                      {"workload": "2D Ising L=8, 16 chains x 10^4 sweeps, 10 graph-captured iterations from ln w = 0"
                                   ", 33 bins, seed 1", "L": L, "chains": P, "sweeps_per_iter": M, "iterations": iters})
    res["iterations_to_flat"] = first_flat or None
    return res


BATCHED_WORKLOAD = "L=16,24,32,48,64 chains=2048 sweeps=100000"


def cpu_baseline_batched(Ls, lnWs, chains, sweeps):
    """The oracle on the host for the batched workload's mix of sizes: one
    thread running `chains` chains of every size for `sweeps` sweeps at the
    weights the GPU reached, then every usable core, each thread running its
    own block of `chains` chains of every size (keyed by the global chain
    index, as a split run is), so that every thread does the same work.  The
    value is the all-core rate; the single-thread rate is kept beside it."""
    import threading

    import oracle as O

    def work(t):
        for L, w in zip(Ls, lnWs):
            O.Run(L, chains, seed=1, bin_shift=1, lnW=w, chain_offset=t * chains).run(sweeps, True)

    per_thread = chains * sweeps * sum(L * L for L in Ls)
    t0 = time.perf_counter()
    work(0)
    dt1 = time.perf_counter() - t0
    T = cpu_threads()
    threads = [threading.Thread(target=work, args=(t,)) for t in range(T)]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    dtT = time.perf_counter() - t0
    return {"value": T * per_thread / dtT, "unit": "spin-flip attempts/s", "cores": T, "kind": "oracle",
            "single_thread_value": per_thread / dt1,
            "sample": "%d threads, each %d chains of every L in %s x %d sweeps at the weights the GPU reached "
                      "(%.3g attempts, %.1f s); single thread: the same %d chains per L (%.1f s)"
                      % (T, chains, Ls, sweeps, T * per_thread, dtT, chains, dt1)}


def bench_batched(a, torch, mc):
    """The batched workload: L in {16, 24, 32, 48, 64}, 2048 chains each, one
    persistent launch per iteration, 10^5 sweeps, the recursion from
    ln w = 0.  Each step replays a HIP graph of one whole iteration (sweeps,
    joints, updates of every size); warmup steps are the first iterations."""
    Ls = BATCHED_LS
    P = a.chains or 2048
    M = a.sweeps or 100000
    sizes = [(L, P, 1, 1) for L in Ls]
    stream = torch.cuda.current_stream()
    ctx = mc.Context(sizes, stream=stream)
    log("bench batched: L=%s, %d chains each, %d sweeps per iteration; autotuning" % (Ls, P, M))
    cpbs = ctx.autotune(200)
    plans = [ctx.launch(i) for i in range(len(Ls))]
    log("bench batched: plans (chains per workgroup, kind, batched) %s" % plans)
    trs = [ctx.new_trace(M, i) for i in range(len(Ls))]
    hs = [ctx.new_hist(i) for i in range(len(Ls))]
    cuts = [ctx.new_cut(i) for i in range(len(Ls))]
    # launch units: (graph, iterations it holds, timed); with --graph-iters G > 1
    # the warmup is one graph of W iterations and the timed steps are graphs of
    # G iterations each (one launch per G steps), else one graph of one
    # iteration is replayed once per step
    gi = max(1, a.graph_iters)
    if a.steps % gi:
        raise SystemExit("--steps must be a multiple of --graph-iters")
    graphs = []
    if gi == 1:
        g1 = ctx.graph(M, 1, trs, hs, cuts)
        graphs.append(g1)
        units = [(g1, 1, s >= a.warmup) for s in range(a.warmup + a.steps)]
    else:
        units = []
        if a.warmup:
            graphs.append(ctx.graph(M, a.warmup, trs, hs, cuts))
            units.append((graphs[-1], a.warmup, False))
        graphs.append(ctx.graph(M, gi, trs, hs, cuts))
        units += [(graphs[-1], gi, True)] * (a.steps // gi)
    metrics = Metrics(a.metrics)
    ev = []
    elapsed = 0.0
    done = 0
    t0 = None
    for g, n_it, timed in units:
        if timed and t0 is None:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.launch()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        done += n_it
        if timed:
            ev += [ms / n_it] * n_it
            elapsed = time.perf_counter() - t0
        for i, L in enumerate(Ls):
            metrics.write(iteration_record(ctx, i, L, P, M, done, ms / n_it))
        log("bench batched: %s step%s %d done (%.0f ms per step%s)"
            % ("timed" if timed else "warmup", "s up to" if n_it > 1 else "", done, ms / n_it,
               ", %.1f s so far" % elapsed if timed else ""))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    metrics.close()
    flats = {str(L): ctx.progress(i)[1] or None for i, L in enumerate(Ls)}
    iters_run = ctx.progress(0)[0]
    weights = [ctx.weights(i) for i in range(len(Ls))]
    att = P * M * sum(L * L for L in Ls)
    for g in graphs:
        g.close()
    ctx.close()
    launch_s = sum(ev) / len(ev) / 1e3
    res = base_record(a, a.steps * att / elapsed, elapsed / a.steps * 1e3,
                      {"workload": "batched uneven L in {16,24,32,48,64}, %d chains each x %d sweeps per iteration "
                                   "in one persistent launch, width-8 energy bins, recursion from ln w = 0, seed 1; "
                                   "one step = one HIP-graph-captured iteration (sweeps + joints + weight updates of "
                                   "every size)%s" % (P, M, "; the timed steps captured %d iterations to a graph"
                                                       % gi if gi > 1 else ""),
                       "L": Ls, "chains_per_L": P, "sweeps_per_iter": M, "parallelism": "chains",
                       "chains_per_block": cpbs, "kernel_kinds": [p_[1] for p_ in plans]})
    res["roofline"] = roofline(att, launch_s, traffic_from_profiles("k_sweep_batched_5L_2048x1e5_counters.md",
                                                                    BATCHED_WORKLOAD))
    res["roofline"]["kernel"] = "k_sweep_batched (mc_run_chains, one persistent launch of the five sizes)"
    res["roofline"]["kernel_ms_basis"] = ("HIP events around each graph replay on the context's stream%s: the sweep "
                                          "launch plus the joints and updates of the five sizes (a few ms)"
                                          % (", divided by the %d iterations it holds" % gi if gi > 1 else ""))
    cc = chain_ceiling(mc, plans[Ls.index(max(Ls))][1], att, M * max(Ls) ** 2)
    if cc is not None:
        cc["frac"] = (att / launch_s) / cc["attempts_per_s"]
        res["roofline"]["chain_ceiling"] = cc
    res["sweep_attempts_per_s"] = att / launch_s
    res["iterations_run"] = iters_run
    res["iterations_to_flat"] = flats
    if not a.no_cpu:
        log("bench batched: timing the CPU oracle on a sample")
        # about 10 s of host work per leg on a current server core
        res["cpu_baseline"] = cpu_baseline_batched(Ls, weights, 4, 4 * a.cpu_sweeps)
    return res


def bench_l128(a, torch, mc):
    """Short runs of a large lattice (--lattice 100, 128 or 256), 8192
    chains x --sweeps (1000) sweeps per step from ln w = 0, for profiling; the
    value is the whole step's rate (run + joint + update)."""
    L, P = a.lattice, a.chains or 8192
    M = a.sweeps or 1000
    stream = torch.cuda.current_stream()
    ctx = mc.Context([(L, P, 1, 1)], stream=stream)
    trace, hist, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
    times = []
    t0 = None
    for s in range(a.warmup + a.steps):
        if s == a.warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.run_chains(M, trace, hist)
        e1.record(stream)
        ctx.join(trace, cut, hist)
        ctx.update_weights(hist, want=False)
        torch.cuda.synchronize()
        if s >= a.warmup:
            times.append(e0.elapsed_time(e1) / 1e3)
        log("bench l128 (L=%d): step %d done" % (L, s + 1))
    elapsed = time.perf_counter() - t0
    att = P * M * L * L
    sweep_s = sum(times) / len(times)
    cpb, kind, _ = ctx.launch()
    ctx.close()
    res = base_record(a, a.steps * att / elapsed, elapsed / a.steps * 1e3,
                      {"workload": "2D Ising L=%d, %d chains x %d sweeps per step (run + joint + update), ln w = 0 "
                                   "start" % (L, P, M),
                       "L": L, "chains": P, "sweeps_per_step": M, "kernel_kind": kind})
    res["roofline"] = roofline(att, sweep_s, None)
    res["roofline"]["kernel"] = kernel_name(kind, L) + " (mc_run_chains)"
    cc = chain_ceiling(mc, kind, att, M * L * L)
    if cc is not None:
        cc["frac"] = (att / sweep_s) / cc["attempts_per_s"]
        res["roofline"]["chain_ceiling"] = cc
    res["sweep_attempts_per_s"] = att / sweep_s
    return res


def bench_large(a, torch, mc):
    """The large-lattice recursion: L = 128 (--lattice), 8192 chains x
    2 x 10^5 sweeps per iteration, from ln w = 0, up to --iters iterations in
    all (40), --steps of them in this call.  Each round is made in --parts
    launches (mc_run_chains_part) with a progress line after each; then the
    joint, the update and the level check (mc_check_levels).  The state is
    checkpointed after every iteration (--state-out) and a later call resumes
    it (--state-in), so the record spans several calls.  The line reports
    this call's iterations; --metrics collects one line per iteration."""
    L = a.lattice
    P = a.chains or 8192
    M = a.sweeps or 200000
    cap = a.iters or 40
    parts = max(1, a.parts)
    if M % parts:
        raise SystemExit("--sweeps must be a multiple of --parts")
    N = L * L
    stream = torch.cuda.current_stream()
    ctx = mc.Context([(L, P, 1, 1)], stream=stream)
    if a.state_in:
        with open(a.state_in, "rb") as f:
            ctx.set_state(f.read())
    done0 = ctx.stats()["updates"]
    todo = min(a.steps, cap - done0)
    cpb, kind, _ = ctx.launch()
    log("bench large: L=%d chains=%d sweeps=%d in %d parts; %d iterations done, %d to run (cap %d); kind %d, "
        "%d chains per workgroup" % (L, P, M, parts, done0, todo, cap, kind, cpb))
    trace, hist, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
    metrics = Metrics(a.metrics)
    sweep_ms, step_s, flat_ratio = [], [], []
    t_all = time.perf_counter()
    for it in range(todo):
        if a.budget_s and step_s and time.perf_counter() - T_START + 1.05 * max(step_s) > a.budget_s:
            log("bench large: the next iteration would pass the time budget; stopping after %d" % it)
            break
        t0 = time.perf_counter()
        ms = 0.0
        for k in range(parts):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.run_chains_part(M // parts, k * (M // parts), trace, hist)
            e1.record(stream)
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            log("bench large: iteration %d, sweeps %d of %d (%.0f s)" % (done0 + it + 1, (k + 1) * (M // parts), M,
                                                                          time.perf_counter() - t0))
        ctx.join(trace, cut, hist)
        ctx.update_weights(hist, want=False)
        ctx.check_levels()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sweep_ms.append(ms)
        step_s.append(dt)
        rec = iteration_record(ctx, 0, L, P, M, done0 + it + 1, dt * 1e3)
        rec["sweep_ms"] = ms
        metrics.write(rec)
        flat_ratio.append(rec["flat_ratio"])
        if a.state_out:
            blob = ctx.get_state()
            with open(a.state_out + ".tmp", "wb") as f:
                f.write(blob)
            os.replace(a.state_out + ".tmp", a.state_out)
        log("bench large: iteration %d done in %.1f s: flat_ratio %.3g, kept %.3f, lnW span %.1f%s"
            % (rec["iteration"], dt, rec["flat_ratio"], rec["retained_frac"], rec["lnW_span"],
               ", FLAT" if rec["flat"] else ""))
        if rec["first_flat"]:
            break
    metrics.close()
    st = ctx.stats()
    ctx.close()
    att = P * M * N
    n = len(sweep_ms)
    elapsed = time.perf_counter() - t_all
    res = base_record(a, n * att / max(elapsed, 1e-9), elapsed / max(n, 1) * 1e3,
                      {"workload": "2D Ising L=%d, %d chains x %d sweeps per iteration, recursion from ln w = 0 to "
                                   "a flat histogram (min h >= 0.8 mean over reachable bins) within %d iterations, "
                                   "width-8 bins, seed 1; iterations %d..%d of the record in this call"
                                   % (L, P, M, cap, done0 + 1, done0 + n),
                       "L": L, "chains": P, "sweeps_per_iter": M, "cap": cap, "kernel_kind": kind,
                       "chains_per_block": cpb})
    res["steps"] = n
    res["warmup"] = 0
    if n:
        sweep_s = sum(sweep_ms) / n / 1e3
        res["roofline"] = roofline(att, sweep_s, None)
        res["roofline"]["kernel"] = kernel_name(kind, L) + " (mc_run_chains_part, %d launches per round)" % parts
        cc = chain_ceiling(mc, kind, att, M * N)
        if cc is not None:
            cc["frac"] = (att / sweep_s) / cc["attempts_per_s"]
            res["roofline"]["chain_ceiling"] = cc
        res["sweep_attempts_per_s"] = att / sweep_s
    res["iterations_done"] = st["updates"]
    res["iterations_to_flat"] = st["first_flat"] or None
    res["flat_ratio_this_call"] = flat_ratio
    return res


def bench_learned256(a, torch, mc):
    """The learned initialiser at L = 256: the network is trained on converged
    weights of L = 8, 16, 32 (recursions from ln w = 0) and 64 (the
    network's own proposal run to flat), then proposes ln w for L = 256;
    4096 chains x --sweeps (2000) sweeps per iteration run from the proposal
    and from ln w = 0 for at most --iters (40) iterations each.  Reported:
    iterations to flat (or none within the cap), the flatness ratio per
    iteration, the difference between the two arms' final ln w, and code
    (ii)'s E, C, F, S of both against Kaufman's exact L = 256 torus."""
    from paper_0812_2964_amd.learned import Initializer, relative_spread, run_to_flat
    import mpmath
    from paper_0812_2964_amd import exact as X

    P, M = a.chains or 4096, a.sweeps or 2000
    cap = a.iters or 40
    Lt = 256
    Nt = Lt * Lt
    t0 = time.perf_counter()
    ini = Initializer(seed=1)
    stages = {}
    for L, c in [(8, 60), (16, 200), (32, 400)]:
        w, flat, done = run_to_flat(L, P, M, c, extra=4)
        stages[L] = {"from": "ln w = 0", "first_flat": flat, "iterations": done}
        if flat is not None:
            ini.add(L, w)
        log("bench learned256: L = %d flat at %s (%.0f s)" % (L, flat, time.perf_counter() - t0))
    ini.fit(steps=4000, lr=2e-3)
    w64, flat, done = run_to_flat(64, P, M, 400, lnW0=ini.predict(64), extra=4)
    stages[64] = {"from": "network (8, 16, 32)", "first_flat": flat, "iterations": done}
    if flat is not None:
        ini.add(64, w64)
    loss = ini.fit(steps=4000, lr=2e-3)
    log("bench learned256: L = 64 flat at %s; trained on %s (loss %.3g, %.0f s)"
        % (flat, [k for k, v in stages.items() if v["first_flat"]], loss, time.perf_counter() - t0))
    if a.stage128:
        t2 = time.perf_counter()

        def progress(done):
            if done % 20 == 0:
                log("bench learned256: L = 128 from the network, %d iterations (%.0f s)"
                    % (done, time.perf_counter() - t2))

        w128, flat, done = run_to_flat(128, P, M, a.stage128, lnW0=ini.predict(128), extra=4, progress=progress)
        stages[128] = {"from": "network (8, 16, 32, 64)", "first_flat": flat, "iterations": done,
                       "seconds": time.perf_counter() - t2}
        if flat is not None:
            ini.add(128, w128)
            loss = ini.fit(steps=4000, lr=2e-3)
        log("bench learned256: L = 128 flat at %s after %d iterations; trained on %s (loss %.3g, %.0f s)"
            % (flat, done, [k for k, v in stages.items() if v["first_flat"]], loss, time.perf_counter() - t0))
    if a.no_arms:
        st128 = stages.get(128)
        att = (st128["iterations"] * P * M * 128 * 128) if st128 else 0
        res = base_record(a, att / st128["seconds"] if st128 else 0.0,
                          st128["seconds"] / max(1, st128["iterations"]) * 1e3 if st128 else 0.0,
                          {"workload": "training stages of the learned initial weight, 4096 chains x %d sweeps per "
                                       "iteration: L = 8, 16, 32 from ln w = 0, 64 and 128 from the network's "
                                       "proposal" % M, "chains": P, "sweeps_per_iter": M})
        res["training"] = {"stages": {str(k): v for k, v in stages.items()}, "loss": loss}
        res["iterations_to_flat"] = {str(k): v["first_flat"] for k, v in stages.items()}
        return res
    metrics = Metrics(a.metrics)
    arms = {}
    finals = {}
    for name, lnW0 in [("learned", ini.predict(Lt)), ("plain", None)]:
        ctx = mc.Context([(Lt, P, 1, 1)])
        ctx.init_weights(lnW0)
        tr, h, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
        t1 = time.perf_counter()
        ratios = []
        for it in range(cap):
            ctx.run_chains(M, tr, h)
            ctx.join(tr, cut, h)
            ctx.update_weights(h, want=False)
            rec = iteration_record(ctx, 0, Lt, P, M, it + 1, 0.0)
            rec["arm"] = name
            metrics.write(rec)
            ratios.append(rec["flat_ratio"])
            log("bench learned256: %s iteration %d: flat_ratio %.3g, lnW span %.0f (%.0f s)"
                % (name, it + 1, rec["flat_ratio"], rec["lnW_span"], time.perf_counter() - t1))
            if rec["first_flat"]:
                break
        st = ctx.stats()
        finals[name] = ctx.weights()
        betas = np.round(np.concatenate([np.arange(0.1, 0.375, 0.05), np.arange(0.40, 0.475, 0.01),
                                         np.arange(0.5, 1.01, 0.1)]), 4)
        e, c, f, s_ = ctx.thermo(betas)
        ctx.close()
        arms[name] = {"iterations_to_flat": st["first_flat"] or None, "iterations_run": st["updates"],
                      "seconds": time.perf_counter() - t1, "flat_ratio": ratios,
                      "thermo": {"beta": betas.tolist(), "E": (e / Nt).tolist(), "C": (c / Nt).tolist(),
                                 "F": (f / Nt).tolist(), "S": (s_ / Nt).tolist()}}
    metrics.close()
    # Kaufman's exact finite-lattice values at the same inverse temperatures
    ex = {"E": [], "C": [], "F": [], "S": []}
    betas = arms["learned"]["thermo"]["beta"]
    with mpmath.workprec(300):
        hh = mpmath.mpf("1e-30")
        for b in betas:
            bb = mpmath.mpf(float(b))
            z0, zp, zm = X.kaufman_lnZ(Lt, bb), X.kaufman_lnZ(Lt, bb + hh), X.kaufman_lnZ(Lt, bb - hh)
            E = -(zp - zm) / (2 * hh)
            ex["E"].append(float(E) / Nt)
            ex["C"].append(float(bb * bb * (zp - 2 * z0 + zm) / (hh * hh)) / Nt)
            ex["F"].append(float(-z0 / bb) / Nt)
            ex["S"].append(float(bb * E + z0) / Nt)
    for name in arms:
        th = arms[name]["thermo"]
        arms[name]["max_abs_dev_per_site"] = {k: float(np.max(np.abs(np.array(th[k]) - np.array(ex[k])))) for k in ex}
    sec = sum(v["seconds"] for v in arms.values())
    att = sum(v["iterations_run"] for v in arms.values()) * P * M * Nt
    res = base_record(a, att / sec, sec / max(1, sum(v["iterations_run"] for v in arms.values())) * 1e3,
                      {"workload": "learned initial weight for L=256, 4096 chains x %d sweeps per iteration, width-8 "
                                   "bins, seed 1, cap %d iterations per arm; network trained on converged ln w of "
                                   "L=%s" % (M, cap, ", ".join(str(k) for k, v in stages.items() if v["first_flat"])),
                       "L": Lt, "chains": P, "sweeps_per_iter": M,
                       "cap": cap})
    res["training"] = {"stages": {str(k): v for k, v in stages.items()}, "loss": loss}
    res["arms"] = arms
    res["exact_per_site"] = ex
    res["iterations_to_flat"] = {k: v["iterations_to_flat"] for k, v in arms.items()}
    res["final_lnW_spread_between_arms"] = relative_spread(finals["learned"], finals["plain"])
    return res


def bench_peaks(a, torch, mc):
    """The microbenchmarks of mc_probe: chip-wide VALU rates of the attempt's
    instruction classes, LDS bandwidth, dependent LDS read latency, a lone
    wave's issue interval, and the quad sweep step alone with and without its
    threshold reads."""
    iters = {0: 4096, 1: 4096, 2: 4096, 3: 2048, 4: 4096, 5: 8192, 6: 1 << 14, 7: 1 << 14, 8: 1 << 14,
             9: 20000, 10: 20000, 11: 20000}
    out = {}
    for k, name in mc.PROBES.items():
        fig, sec, work, cyc = mc.probe(k, iters[k])
        out[name] = {"value": fig, "seconds": sec, "work": work, "cycles": cyc}
        log("bench peaks: %s = %.4g (%.3f ms)" % (name, fig, sec * 1e3))
    res = base_record(a, out["valu_xor"]["value"], out["valu_xor"]["seconds"] * 1e3,
                      {"workload": "mc_probe microbenchmarks (chip-wide VALU rates, LDS bandwidth and latency, "
                                   "lone-wave issue interval)"})
    res["metric"] = "32-bit VALU lane-instructions/s (v_xor_b32), with the other probes beside it"
    res["unit"] = "lane-instructions/s"
    res["probes"] = out
    res["derived"] = {
        "valu_peak_spec": ALU_PEAK_OPS,
        "valu_xor_frac_of_spec": out["valu_xor"]["value"] / ALU_PEAK_OPS,
        "mul_lo_rate_vs_xor": out["valu_mul_lo"]["value"] / out["valu_xor"]["value"],
        "mul_hi_rate_vs_xor": out["valu_mul_hi"]["value"] / out["valu_xor"]["value"],
        "mad_u64_rate_vs_xor": out["valu_mad_u64"]["value"] / out["valu_xor"]["value"],
        "lds_bytes_per_clk_per_cu": out["lds_read_bandwidth"]["value"] / (256 * CLOCK_HZ),
        "quad_step_cycles_per_attempt": out["quad_step_cycles"]["value"] / 4.0,
        "quad_step_share_of_threshold_reads": 1.0 - out["quad_step_cycles_no_threshold_reads"]["value"]
                                              / out["quad_step_cycles"]["value"],
        "shader_clock_hz_seen_by_lone_wave_probe": out["lone_wave_independent_issue_cycles"]["cycles"]
                                                   / out["lone_wave_independent_issue_cycles"]["seconds"]}
    return res


def bench_thermo(a, torch, mc):
    """Reduced reweighting (mc_thermo, the paper's code (ii)) at L = 256:
    E, C, F, S at n_beta inverse temperatures from a smooth synthetic weight of
    32769 bins (65535 reachable levels)."""
    L = 256
    N = L * L
    nb = (N >> 1) + 1
    n_beta = a.chains or 4096
    rng = np.random.default_rng(1)
    x = (np.arange(nb) - nb / 2) / nb
    w = -0.6 * N * x * x + np.cumsum(rng.normal(0, 0.05, nb))
    betas = np.linspace(0.05, 2.0, n_beta)
    ctx = mc.Context([(L, 2, 1, 1)])
    ctx.init_weights(w)
    for _ in range(a.warmup):
        ctx.thermo(betas)
    times = []
    for _ in range(a.steps):
        t0 = time.perf_counter()
        ctx.thermo(betas)
        times.append(time.perf_counter() - t0)
    ctx.close()
    dt = sum(times) / len(times)
    terms = n_beta * (N - 1)
    res = base_record(a, terms / dt, dt * 1e3,
                      {"workload": "reduced reweighting at L=256: E, C, F, S at %d inverse temperatures from a "
                                   "synthetic weight of 32769 bins" % n_beta, "L": L, "n_beta": n_beta},
                      dtype="f64")
    res["metric"] = "reweighting terms/s (inverse temperature x energy level)"
    res["unit"] = "terms/s"
    # per term, as the kernel evaluates it: two exponentials (about 12 fp64
    # operations each; each term's is taken once for Z and the mean and once for
    # the variance) and 10 additions and multiplications
    flops = 34.0 * terms / dt
    res["roofline"] = {"bound": "alu", "achieved": flops / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                       "frac": flops / 78.6e12, "traffic": None, "kernel": "k_thermo (mc_thermo, incl. copies)"}
    if not a.no_cpu:
        from oracle.thermo import thermo as o_thermo

        sb = betas[:: 4]
        t0 = time.perf_counter()
        o_thermo(w, L, 1, sb)
        tc = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": len(sb) * (N - 1) / tc, "unit": "terms/s", "cores": 1, "kind": "oracle",
                               "sample": "%d of the inverse temperatures (%.2f s, numpy, single thread)"
                                         % (len(sb), tc)}
    return res


def bench_fig2(a, torch, mc):
    """The comparison of Fig. 2 (Sec. 5): multicanonical weights generated with
    detailed-balance joints (mode 0) and with naive splices (mode 1), then the
    energy of code (ii) against Kaufman's exact energy of the L = 20 torus.
    Each iteration collects about 10^8 attempts (M_total) in rounds of
    32 chains x 100 sweeps (M_node), joined after every round (Algorithm
    step 6), before the weight update; one bin per level, so that the energy
    resolution of the weight is that of the model."""
    from paper_0812_2964_amd import exact as X

    L, P, M = 20, a.chains or 32, a.sweeps or 100
    N = L * L
    rounds = a.rounds or max(1, round(1e8 / (P * M * N)))
    iters = a.iters or 200
    betas = np.round(np.linspace(0.05, 1.0, 20), 4)
    exact = np.array([X.mean_energy_exact(L, b) for b in betas])
    res = base_record(a, 0.0, 0.0, {"workload": "Fig. 2 comparison: L=20, %d chains x %d sweeps per round, %d "
                                                "rounds per iteration, %d iterations from ln w = 0, one bin per "
                                                "level, seed 1" % (P, M, rounds, iters),
                                    "L": L, "chains": P, "sweeps_per_round": M, "rounds_per_iteration": rounds,
                                    "iterations": iters})
    res["metric"] = METRIC
    total_att, total_s = 0, 0.0
    res["modes"] = {}
    for mode in (0, 1):
        ctx = mc.Context([(L, P, 1, 0)])
        tr, h, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kept = 0
        for it in range(iters):
            for _ in range(rounds):
                ctx.run_chains(M, tr, h)
                ctx.join(tr, cut, h, mode)
            ctx.update_weights(h, want=False)
            if (it + 1) % 50 == 0:
                torch.cuda.synchronize()
                log("bench fig2: mode %d, iteration %d (%.1f s)" % (mode, it + 1, time.perf_counter() - t0))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        upd, first_flat, _, kept = ctx.progress()
        e = ctx.thermo(betas)[0]
        ctx.close()
        dev = (e - exact) / N
        hi = betas < 0.35
        total_att += iters * rounds * P * M * N
        total_s += dt
        res["modes"]["detailed_balance" if mode == 0 else "naive"] = {
            "first_flat_iteration": first_flat or None,
            "kept_fraction_last_iteration": kept / float(rounds * P * M),
            "max_abs_dE_per_site_beta_lt_0.35": float(np.max(np.abs(dev[hi]))),
            "max_abs_dE_per_site_beta_ge_0.35": float(np.max(np.abs(dev[~hi]))),
            "dE_per_site": {str(b): float(d) for b, d in zip(betas, dev)},
            "seconds": dt}
    res["value"] = total_att / total_s
    res["ms_per_step"] = total_s / (2 * iters) * 1e3
    return res


def bench_topup(a, torch, mc):
    """Algorithm step 6 with the energy ordering of Sec. 2's remark: the Fig. 2
    setting (L = 20, 32 chains, one bin per level, seed 1, from ln w = 0), but
    each iteration is mc_iterate_topup: rounds of at most M_node = 100 sweeps
    until M_total = 2.5e5 configurations (10^8 attempts) are kept.  Joints in
    chain order (mode 0), in energy order (mode 2) and the naive splice
    (mode 1) are compared by retention, rounds and sweeps per iteration,
    iterations to the first flat histogram and the energy of code (ii) against
    Kaufman's exact energy of the 20 x 20 torus."""
    from paper_0812_2964_amd import exact as X

    L, P, M = 20, a.chains or 32, a.sweeps or 100
    N = L * L
    m_total = int(round(1e8 / N))
    iters = a.iters or 200
    betas = np.round(np.linspace(0.05, 1.0, 20), 4)
    exact = np.array([X.mean_energy_exact(L, b) for b in betas])
    res = base_record(a, 0.0, 0.0, {"workload": "Algorithm step 6: L=20, %d chains, rounds of at most %d sweeps "
                                                "until %d configurations are kept, %d iterations from ln w = 0, "
                                                "one bin per level, seed 1" % (P, M, m_total, iters),
                                    "L": L, "chains": P, "max_sweeps_per_round": M, "m_total": m_total,
                                    "iterations": iters})
    total_att, total_s = 0, 0.0
    res["modes"] = {}
    for mode, name in ((0, "detailed_balance_chain_order"), (2, "detailed_balance_energy_order"), (1, "naive")):
        ctx = mc.Context([(L, P, 1, 0)])
        tr, h, cut = ctx.new_trace(M), ctx.new_hist(), ctx.new_cut()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for it in range(iters):
            stats.append(ctx.iterate_topup(m_total, M, tr, h, cut, mode=mode))
            if (it + 1) % 50 == 0:
                log("bench topup: mode %d, iteration %d (%.1f s)" % (mode, it + 1, time.perf_counter() - t0))
        dt = time.perf_counter() - t0
        _, first_flat, _, _ = ctx.progress()
        e = ctx.thermo(betas)[0]
        ctx.close()
        rounds = np.array([s_[0] for s_ in stats])
        sweeps = np.array([s_[1] for s_ in stats])
        kept = np.array([s_[2] for s_ in stats])
        gen = sweeps * P
        dev = (e - exact) / N
        hi = betas < 0.35
        total_att += int(gen.sum()) * N
        total_s += dt
        res["modes"][name] = {
            "first_flat_iteration": first_flat or None,
            "retention_all": float(kept.sum() / gen.sum()),
            "retention_last_50": float(kept[-50:].sum() / gen[-50:].sum()),
            "rounds_per_iteration_mean": float(rounds.mean()),
            "sweeps_per_iteration_last_50": float(sweeps[-50:].mean()),
            "generated_per_kept_last_50": float(gen[-50:].sum() / kept[-50:].sum()),
            "max_abs_dE_per_site_beta_lt_0.35": float(np.max(np.abs(dev[hi]))),
            "max_abs_dE_per_site_beta_ge_0.35": float(np.max(np.abs(dev[~hi]))),
            "seconds": dt}
    res["value"] = total_att / total_s
    res["ms_per_step"] = total_s / (3 * iters) * 1e3
    return res


def bench_fig1(a, torch, mc):
    """The comparison of Fig. 1 (Sec. 5) at the paper's L = 100 (and L = 64):
    E/N, C, F/N and S/N from code (ii) against the exact finite-lattice values
    (Kaufman's ln Z and its beta derivatives).  The weight comes from the
    learned initialiser instead of 1300 iterations: converged weights of
    L = 8, 16, 32 (recursions from ln w = 0) train the network, its proposal
    for L = 64 is run to flat, the network is trained again with L = 64 added,
    and its proposal for L = 100 is run to flat (at most --iters
    iterations)."""
    from paper_0812_2964_amd.learned import Initializer, run_to_flat
    import mpmath
    from paper_0812_2964_amd import exact as X

    P, M = a.chains or 4096, a.sweeps or 2000
    P_big = 8192
    cap = a.iters or 150
    L = 100
    N = L * L
    t0 = time.perf_counter()
    ini = Initializer(seed=1)
    stages, att = {}, 0
    for Ls, c in [(8, 60), (16, 200), (32, 400)]:
        w, flat, done = run_to_flat(Ls, P, M, c, extra=4)
        stages[Ls] = {"from": "ln w = 0", "first_flat": flat, "iterations": done}
        att += done * P * M * Ls * Ls
        if flat is not None:
            ini.add(Ls, w)
    ini.fit(steps=4000, lr=2e-3)
    log("bench fig1: trained on L = 8, 16, 32 (%.1f s)" % (time.perf_counter() - t0))
    w64, flat, done = run_to_flat(64, P, M, cap, lnW0=ini.predict(64), extra=4)
    stages[64] = {"from": "network (8, 16, 32)", "first_flat": flat, "iterations": done}
    att += done * P * M * 64 * 64
    if flat is not None:
        ini.add(64, w64)
        ini.fit(steps=4000, lr=2e-3)
    log("bench fig1: L = 64 flat at %s, retrained (%.1f s)" % (flat, time.perf_counter() - t0))
    wL, flat, done = run_to_flat(L, P_big, M, cap, lnW0=ini.predict(L), extra=4,
                                 progress=lambda d: log("bench fig1: L = %d, %d iterations" % (L, d))
                                 if d % 20 == 0 else None)
    stages[L] = {"from": "network (8, 16, 32, 64)", "first_flat": flat, "iterations": done, "chains": P_big}
    att += done * P_big * M * N
    dt = time.perf_counter() - t0
    if a.out_npz:
        np.savez(a.out_npz, lnW64=w64, lnW100=wL)
    betas = np.round(np.concatenate([np.arange(0.1, 0.375, 0.05), np.arange(0.40, 0.475, 0.01),
                                     np.arange(0.5, 1.01, 0.1)]), 4)

    def compare(Ls, w):
        Ns = Ls * Ls
        ctx = mc.Context([(Ls, 2, 1, 1)])
        ctx.init_weights(w)
        e, c, f, s_ = ctx.thermo(betas)
        ctx.close()
        ex = {"E": [], "C": [], "F": [], "S": []}
        with mpmath.workprec(300):
            h = mpmath.mpf("1e-30")
            for b in betas:
                bb = mpmath.mpf(float(b))
                z0, zp, zm = X.kaufman_lnZ(Ls, bb), X.kaufman_lnZ(Ls, bb + h), X.kaufman_lnZ(Ls, bb - h)
                E = -(zp - zm) / (2 * h)
                ex["E"].append(float(E))
                ex["C"].append(float(bb * bb * (zp - 2 * z0 + zm) / (h * h)))
                ex["F"].append(float(-z0 / bb))
                ex["S"].append(float(bb * E + z0))
        ex = {k: np.array(v) for k, v in ex.items()}
        got = {"E": e, "C": c, "F": f, "S": s_}
        return {"per_site": {k: (v / Ns).tolist() for k, v in got.items()},
                "exact_per_site": {k: (v / Ns).tolist() for k, v in ex.items()},
                "max_abs_dev_per_site": {k: float(np.max(np.abs(got[k] - ex[k])) / Ns) for k in got},
                "max_rel_dev_C": float(np.max(np.abs(c - ex["C"]) / ex["C"])),
                "C_peak": {"beta_exact": float(betas[np.argmax(ex["C"])]), "beta": float(betas[np.argmax(c)]),
                           "C_per_site_exact": float(ex["C"].max() / Ns), "C_per_site": float(c.max() / Ns)}}

    res = base_record(a, att / dt, dt * 1e3,
                      {"workload": "Fig. 1 comparison at L=%d (and L=64): learned initial weight (network trained on "
                                   "converged ln w of L=8, 16, 32, then 64), recursion to flat with %d chains x %d "
                                   "sweeps per iteration, width-8 bins, seed 1, cap %d; code (ii) against the exact "
                                   "finite lattice" % (L, P_big, M, cap), "L": L, "chains": P_big,
                       "sweeps_per_iter": M, "cap": cap})
    res["stages"] = {str(k): v for k, v in stages.items()}
    res["betas"] = betas.tolist()
    res["L64"] = compare(64, w64)
    res["L%d" % L] = compare(L, wL)
    return res


def bench_learned(a, torch, mc):
    """The learned initial weight: the network is trained on converged weights
    of L = 8, 16 and 32, and proposes the weight of L = 64; iterations to the
    first flat histogram from that proposal against the recursion from
    ln w = 0 (w^(1) = 1), with the same chains, sweeps and seed."""
    from paper_0812_2964_amd.learned import Initializer, run_to_flat

    P, M = a.chains or 4096, a.sweeps or 2000
    cap = a.iters or 500
    target = 64
    t0 = time.perf_counter()
    ini = Initializer(seed=1)
    train = {}
    for L, c in [(8, 60), (16, 200), (32, 400)]:
        w, flat, done = run_to_flat(L, P, M, c, extra=4,
                                    progress=lambda d, L=L: log("bench learned: L=%d, %d iterations" % (L, d))
                                    if d % 40 == 0 else None)
        train[L] = flat
        if flat is not None:
            ini.add(L, w)
    loss = ini.fit(steps=4000, lr=2e-3)
    t_train = time.perf_counter() - t0
    log("bench learned: trained (loss %.3g) in %.1f s" % (loss, t_train))
    runs = {}
    for name, lnW0 in [("learned", ini.predict(target)), ("plain", None)]:
        t1 = time.perf_counter()
        _, flat, done = run_to_flat(target, P, M, cap, lnW0=lnW0,
                                    progress=lambda d, n=name: log("bench learned: L=%d %s, %d iterations"
                                                                   % (target, n, d)) if d % 40 == 0 else None)
        runs[name] = {"iterations_to_flat": flat, "iterations_run": done, "seconds": time.perf_counter() - t1}
    att = sum(r["iterations_run"] for r in runs.values()) * P * M * target * target
    sec = sum(r["seconds"] for r in runs.values())
    res = base_record(a, att / sec, sec / max(1, sum(r["iterations_run"] for r in runs.values())) * 1e3,
                      {"workload": "learned initial weight for L=%d: network trained on converged ln w of L=8, 16, 32 "
                                   "(%d chains x %d sweeps per iteration, width-8 bins, seed 1), iterations to flat "
                                   "against ln w = 0, cap %d" % (target, P, M, cap),
                       "L": target, "chains": P, "sweeps_per_iter": M, "cap": cap})
    res["training"] = {"first_flat": train, "loss": loss, "seconds": t_train}
    res["iterations_to_flat"] = {k: v["iterations_to_flat"] for k, v in runs.items()}
    res["runs"] = runs
    return res


def bench_copy(a, torch):
    """A plain device-to-device copy of known size (counter calibration)."""
    n = a.copy_bytes // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"copy_bytes": n * 4, "copies": 3}


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the chains of one ensemble live on a single device here "
              "(sharding across GPUs is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if a.workload == "batched" and (a.graph_iters < 1 or a.steps % a.graph_iters):
        print("bench.py: --steps (%d) must be a multiple of --graph-iters (%d >= 1)" % (a.steps, a.graph_iters),
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_0812_2964_amd as mc

    torch.cuda.set_device(0)
    if a.workload == "copy":
        res = bench_copy(a, torch)
    elif a.workload == "recursion8":
        res = bench_recursion8(a, torch, mc)
    elif a.workload == "batched":
        res = bench_batched(a, torch, mc)
    elif a.workload == "l128":
        res = bench_l128(a, torch, mc)
    elif a.workload == "large":
        res = bench_large(a, torch, mc)
    elif a.workload == "learned256":
        res = bench_learned256(a, torch, mc)
    elif a.workload == "peaks":
        res = bench_peaks(a, torch, mc)
    elif a.workload == "thermo":
        res = bench_thermo(a, torch, mc)
    elif a.workload == "fig2":
        res = bench_fig2(a, torch, mc)
    elif a.workload == "topup":
        res = bench_topup(a, torch, mc)
    elif a.workload == "fig1":
        res = bench_fig1(a, torch, mc)
    elif a.workload == "learned":
        res = bench_learned(a, torch, mc)
    elif a.workload == "l32":
        res = bench_l32(a, torch, mc)
    else:
        res = bench_batched(a, torch, mc)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
