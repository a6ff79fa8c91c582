"""Compile the HIP library (libmcgpu.so) for gfx950 with hipcc.

Flags:
  -ffp-contract=off    every fused multiply-add in the binary64 code is written
                       out, so thresholds and weights are reproducible bit for bit;
  -packed-fp32-ops     the gfx950 target feature turned off, so the device pass
                       generates no packed fp32 instructions (v_pk_fma_f32 and
                       the like).  hipcc hands the flag to the host (x86) pass
                       too, which does not know the feature and warns that it
                       ignores it; that warning is dropped from the output
                       below, everything else the compiler prints is shown.
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
# what the host pass prints for the device-only target feature above
HOST_FEATURE_WARNING = "'-packed-fp32-ops' is not a recognized feature for this target"


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
    """Compile every source to an object (in parallel) under _build/, then
    link the shared library; the library is replaced only when both succeed."""
    from concurrent.futures import ThreadPoolExecutor

    obj_dir = os.path.join(ROOT, "_build", "mcgpu")
    os.makedirs(obj_dir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
        jobs.append(([hipcc()] + compile_flags() + list(extra) + ["-c", "-o", obj, os.path.join(CSRC, src)], obj))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        out = "\n".join(l for l in p.stdout.splitlines() if HOST_FEATURE_WARNING not in l)
        if out.strip():
            print(out, flush=True)
        if p.returncode != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)

    with ThreadPoolExecutor(max_workers=min(len(jobs), max(1, (os.cpu_count() or 1)))) as ex:
        for f in [ex.submit(run, cmd) for cmd, _ in jobs]:
            f.result()
    run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", LIB + ".tmp"] + [obj for _, obj in jobs])
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
