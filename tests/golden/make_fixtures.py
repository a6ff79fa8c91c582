"""Write the stored inputs of the GPU parity tests and the benchmark.

Every value is produced by the CPU oracle (oracle/), nothing else:

  lnW_L32_prior.npy  ln w (513 width-8 bins, binary64) of the L = 32 lattice
                     after 30 iterations of the multicanonical recursion
                     (Sec. 3.1 eq. new_weight, run as in Sec. 4.2): 32 chains,
                     2000 sweeps per iteration, seed 1, ln w = 0 start.  It is
                     the "fixed ln w from a prior iteration" of the L = 32,
                     4096-chain workload.

Run:  python tests/golden/make_fixtures.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402


def lnw_L32_prior(iters=30, chains=32, sweeps=2000):
    R = O.Run(32, chains, seed=1, bin_shift=1)
    for it in range(iters):
        tr, _ = R.run(sweeps)
        R.join(tr)
        flat = R.update()
        print("iteration %d: visited bins %d, flat %s" % (it + 1, int((R.lnW != 0).sum()), flat), flush=True)
    return R.lnW


def main():
    w = lnw_L32_prior()
    path = os.path.join(HERE, "lnW_L32_prior.npy")
    np.save(path, w)
    print(path, hashlib.sha256(open(path, "rb").read()).hexdigest())


if __name__ == "__main__":
    main()
