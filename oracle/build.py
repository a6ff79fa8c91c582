"""Build the CPU oracle (test infrastructure) as a shared library with gcc.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
load the result.  Flags: no contraction of a*b+c into fma (every fma in the
oracle is written out), no fast-math, so each binary64 operation rounds once
as IEEE-754 prescribes.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["mc_oracle.c", "mlp_oracle.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-Werror", "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
