"""Host logic of the benchmark script (no GPU): the multi-core oracle leg of
its CPU baseline splits the chains into contiguous blocks keyed by their global
index, which is the same computation as one run over all of them; the
`--gpus` guard; the traffic figure is only taken from a counter summary of the
current kernel source and workload."""
import os
import subprocess
import sys
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402


def test_threaded_blocks_equal_one_run():
    import bench

    L, blk, T, M = 8, 3, 4, 25
    w = np.random.default_rng(3).normal(0, 2.0, O.n_bins(L, 1))
    whole = O.Run(L, T * blk, seed=1, bin_shift=1, lnW=w)
    tr, h = whole.run(M)
    runs = [O.Run(L, blk, seed=1, bin_shift=1, lnW=w, chain_offset=t * blk) for t in range(T)]
    out = [None] * T

    def go(t):
        out[t] = runs[t].run(M)

    ths = [threading.Thread(target=go, args=(t,)) for t in range(T)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    assert np.array_equal(np.concatenate([o[0] for o in out]), tr)
    assert np.array_equal(sum(o[1] for o in out), h)
    assert np.array_equal(np.concatenate([r.spins for r in runs]), whole.spins)
    assert 1 <= bench.cpu_threads() <= 16
    cb = bench.cpu_baseline(L, w, 4, 20)
    assert cb["kind"] == "oracle" and cb["cores"] == bench.cpu_threads() and cb["value"] > 0


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0 and "one GPU" in (p.stdout + p.stderr)


def test_graph_iterations_must_divide_the_steps():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--graph-iters", "3", "--steps", "4"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "multiple of --graph-iters" in p.stderr


def test_traffic_only_for_current_source_and_workload(tmp_path, monkeypatch):
    """A counter summary is used only when its kernel source hash and its
    workload line match."""
    import bench

    prof = tmp_path / "profiles"
    prof.mkdir()
    h = bench.kernel_source_hash()
    (prof / "x.md").write_text("workload: L=32 chains=4096 sweeps=100000\nkernel source sha256: %s\n"
                               "HBM bytes per launch (scaled): 8.21e+08\n" % h)
    (prof / "old.md").write_text("workload: L=32 chains=4096 sweeps=100000\nkernel source sha256: %s\n"
                                 "HBM bytes per launch (scaled): 8.21e+08\n" % ("0" * 64))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.traffic_from_profiles("x.md", "L=32 chains=4096 sweeps=100000") == 8.21e8
    assert bench.traffic_from_profiles("x.md", "L=32 chains=4096 sweeps=99999") is None
    assert bench.traffic_from_profiles("old.md", "L=32 chains=4096 sweeps=100000") is None
    assert bench.traffic_from_profiles("missing.md", "L=32 chains=4096 sweeps=100000") is None


def test_batched_cpu_baseline_and_iteration_record():
    """The batched workload's oracle leg runs every size on every thread; the
    per-iteration record derives its fields from mc_get_stats."""
    import bench

    Ls = [4, 6]
    cb = bench.cpu_baseline_batched(Ls, [np.zeros(O.n_bins(L, 1)) for L in Ls], 2, 5)
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] == bench.cpu_threads()

    class FakeCtx:
        def stats(self, i):
            return {"updates": 3, "retained_last": 150, "join_none": 2, "join_cut_sum": 30, "join_cut_max": 9,
                    "hist_min": 10, "n_reach_bins": 5, "hist_sum": 100, "last_flat": 0, "first_flat": 0,
                    "lnw_min": -4.0, "lnw_max": 1.5}

    r = bench.iteration_record(FakeCtx(), 0, 8, 10, 20, 3, 12.5)
    assert r["retained_frac"] == 150 / 200.0 and r["n_no_accept"] == 2 and r["mean_cut"] == 30 / 8.0
    assert r["max_cut"] == 9 and r["flat_ratio"] == 0.5 and r["lnW_span"] == 5.5 and r["first_flat"] is None


def test_record_carries_the_contract_keys():
    """The JSON line's keys and the roofline object's arithmetic, without a
    GPU: frac = achieved / peak, achieved = ops per attempt x attempts / the
    kernel's time, the peak from 256 CUs x 128 lanes x 2.4 GHz."""
    import argparse

    import bench

    a = argparse.Namespace(steps=3, warmup=1)
    rec = bench.base_record(a, 1.0e11, 3500.0, {"workload": "x"})
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config"):
        assert k in rec, k
    assert rec["n_gpus"] == 1 and rec["vs_baseline"] is None and rec["config"]["workload"] == "x"
    r = bench.roofline(4.194304e11, 3.5, 8.2e8)
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["bound"] == "alu" and r["traffic"] == 8.2e8
    assert abs(r["peak"] - 256 * 128 * 2.4e9 / 1e12) < 1e-9
    assert abs(r["achieved"] - 31 * 4.194304e11 / 3.5 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12


def test_chain_ceiling_from_the_issue_interval():
    """The chain ceiling of a launch: the longest chain issues valu_per_step
    instructions per four sites at one per issue interval, so a launch of A
    attempts whose longest chain makes S of them takes at least
    S x valu x interval / 4 cycles.  A stub stands in for the probe."""
    import bench

    class Probe:
        def probe(self, kind, iters):
            assert kind == 8
            return 4.0, 1.0, 0, 2.4e9  # 4 cycles per instruction; a 2.4 GHz clock over 1 s

    A, S = 1.0e12, 4.0e8
    cc = bench.chain_ceiling(Probe(), 7, A, S)
    floor = bench.CONSUMER_VALU_PER_STEP[7] * 4.0 / 4.0
    assert cc["cycles_per_attempt_floor"] == floor and cc["kernel_kind"] == 7
    assert abs(cc["attempts_per_s"] - A / (S * floor / bench.CLOCK_HZ)) <= 1e-9 * cc["attempts_per_s"]
    assert abs(cc["probe_clock_hz"] - 2.4e9) < 1.0
    assert bench.chain_ceiling(Probe(), 3, A, S) is None  # the bit-by-bit kind has no counted step
