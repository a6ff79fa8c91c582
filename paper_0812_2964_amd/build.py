"""Compile the HIP library (libmcgpu.so) for gfx950 with hipcc.

Flags:
  -ffp-contract=off    every fused multiply-add in the binary64 code is written
                       out, so thresholds and weights are reproducible bit for bit;
  -packed-fp32-ops off no packed fp32 instructions are generated.
"""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["mc_kernels.hip", "mc_api.hip", "mc_mlp.hip", "mc_thermo.hip", "mc_probe.hip"]
LIB = os.path.join(HERE, "libmcgpu.so")
ARCH = os.environ.get("MCGPU_ARCH", "gfx950")


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def compile_flags():
    return ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build(verbose: bool = False, extra=()) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [hipcc()] + compile_flags() + list(extra) + ["-shared", "-o", LIB + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
