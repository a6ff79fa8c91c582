"""Pins of the oracle's elementary pieces: Philox4x32-10, exp, log, thresholds.

* Philox is compared word for word with rocRAND's independent implementation
  of the same generator (its public header, called from a small host program
  built with hipcc at test time), on counters spanning all four words.
* exp/log are compared with the C library and with 300-bit mpmath.
* The acceptance threshold is compared with its closed form.
"""
import math
import os
import shutil
import subprocess
import tempfile

import mpmath
import numpy as np
import pytest

import oracle as O

KAT_SRC = r"""
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c[4], k[2];
  while (scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
    unsigned long long sub = ((unsigned long long)c[3] << 32) | c[2];
    unsigned long long off = (((unsigned long long)c[1] << 32) | c[0]) * 4ull; /* c[1] < 2^30 */
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 r = e.next4();
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


def _rocrand_philox(rows):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "kat.cpp")
        exe = os.path.join(d, "kat")
        open(src, "w").write(KAT_SRC)
        subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
        inp = "\n".join(" ".join("%08x" % v for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]


def test_philox_matches_rocrand():
    rng = np.random.default_rng(12345)
    rows = [[0, 0, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0], [0, 1, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0], [0, 0, 0, 1, 0, 0],
            [0, 0, 0, 0, 1, 0], [0, 0, 0, 0, 0, 1], [0xFFFFFFFF, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]]
    for _ in range(200):
        r = [int(x) for x in rng.integers(0, 2**32, size=6)]
        r[1] &= (1 << 30) - 1
        rows.append(r)
    ref = _rocrand_philox(rows)
    assert len(ref) == len(rows)
    for r, want in zip(rows, ref):
        got = O.philox(r[:4], r[4:])
        assert [int(x) for x in got] == want, r


def test_uniform_word_selection_and_keying():
    # word j&3 of the block with counter word 0 = j>>2 (reading R4)
    seed, L = 7, 32
    for dom, a, c, j in [(0, 5, 3, 0), (0, 5, 3, 1), (0, 5, 3, 2), (0, 5, 3, 3), (1, 0, 9, 1023), (2, 4, 1, 77)]:
        blk = O.philox([j >> 2, a, c, dom], [seed, L])
        assert O.uniform(seed, L, dom, a, c, j) == int(blk[j & 3])
    # the lattice size is part of the key: different L, different stream
    assert O.uniform(1, 16, 0, 0, 0, 0) != O.uniform(1, 24, 0, 0, 0, 0)


def test_uniform_is_uniform():
    # chi-square over 64 cells of 2^16 words of one sweep stream
    words = np.array([O.uniform(1, 32, 0, 3, 11, j) for j in range(1 << 16)], dtype=np.uint64)
    cells = np.bincount((words >> np.uint64(26)).astype(np.int64), minlength=64)
    e = len(words) / 64
    chi2 = ((cells - e) ** 2 / e).sum()
    assert chi2 < 120  # dof 63; p(chi2 > 120) ~ 1e-5


def _ulp_diff(a, b):
    ia = np.frombuffer(np.float64(a).tobytes(), dtype=np.int64)[0]
    ib = np.frombuffer(np.float64(b).tobytes(), dtype=np.int64)[0]
    return abs(int(ia) - int(ib))


def test_det_exp_accuracy():
    rng = np.random.default_rng(1)
    xs = np.concatenate([-rng.uniform(0, 23, 20000), -rng.uniform(0, 1e-3, 2000), -np.logspace(-12, 2.8, 500),
                         [0.0, -math.log(2), -1.0, -22.9, -700.0]])
    worst = 0
    for x in xs:
        worst = max(worst, _ulp_diff(O.det_exp(x), math.exp(x)))
    assert worst <= 1
    with mpmath.workprec(300):
        for x in xs[::50]:
            exact = float(mpmath.exp(mpmath.mpf(float(x))))
            assert _ulp_diff(O.det_exp(x), exact) <= 1
    assert O.det_exp(0.0) == 1.0
    assert O.det_exp(-800.0) == 0.0


def test_det_log_accuracy():
    rng = np.random.default_rng(2)
    hs = np.concatenate([np.arange(1, 5000), rng.integers(1, 2**31, 20000), [2**k for k in range(31)],
                         [2**31 - 1, 3 * 2**20, 46341]])
    worst = 0
    for h in hs:
        worst = max(worst, _ulp_diff(O.det_log(int(h)), math.log(int(h))))
    assert worst <= 1
    assert O.det_log(1) == 0.0
    with mpmath.workprec(300):
        for h in hs[::97]:
            assert _ulp_diff(O.det_log(int(h)), float(mpmath.log(int(h)))) <= 1


def test_threshold_closed_form():
    assert O.threshold(0.0) == 0xFFFFFFFF
    assert O.threshold(3.5) == 0xFFFFFFFF
    assert O.threshold(-24.0) == 0
    assert O.threshold(-23.0001) == 0
    # exact halving: exp(-ln 2) * 2^32 = 2^31 up to one ulp of the exponential
    assert O.threshold(-math.log(2.0)) in (2**31 - 1, 2**31)
    rng = np.random.default_rng(3)
    prev = -1
    for d in np.sort(-rng.uniform(0, 23, 3000)):
        t = O.threshold(d)
        want = math.floor(math.exp(d) * 2.0**32)
        assert abs(t - min(want, 2**32 - 1)) <= 1
        assert t >= prev  # monotone in d
        prev = t
    # acceptance probability (tau + 1) / 2^32: tau = 2^32 - 1 always accepts
    assert O.threshold(-1e-12) == 0xFFFFFFFF
