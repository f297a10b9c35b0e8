"""Build the HIP library of the DSMC hot path for gfx950 (in-tree).

The library is compiled with hipcc directly (no torch extension): plain
C ABI, loaded with ctypes by ``binding.py``.  Floating-point flags matter for
the method's reproducibility: no contraction of multiply-adds
(``-ffp-contract=off``), correctly rounded FP32 division and square root,
and no packed-FP32 instructions.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libdsmc_hip.so")
# the same sources with kernel index checks (-DDSMC_BOUNDS_CHECK): failed
# checks are counted in dsmc_diag.bounds_violations; for tests
LIB_BOUNDS = os.path.join(OUT_DIR, "libdsmc_hip_bounds.so")
SOURCES = ["dsmc_api.hip", "dsmc_mlp.hip"]
HEADERS = ["dsmc_device.h", "dsmc_kernels.h", "dsmc_collide.h", "dsmc_learned.h",
           "dsmc_collide_kernels.h"]
ARCH = os.environ.get("DSMC_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    "-ffp-contract=off",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, bounds=True):
    """Compile every HIP source into the in-tree shared library and, unless
    bounds is False, the bounds-checking variant beside it (both at once;
    always rebuilds).  Returns the release library's path."""
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = []
    for out, extra in ((LIB, []), (LIB_BOUNDS, ["-DDSMC_BOUNDS_CHECK"])):
        if out == LIB_BOUNDS and not bounds:
            continue
        tmp = out + ".tmp%d" % os.getpid()
        cmd = [hipcc(), *FLAGS, *extra, "-I", os.path.join(ROOT, "include"),
               *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((subprocess.Popen(cmd), tmp, out, cmd))
    failed = None
    for proc, tmp, out, cmd in jobs:
        if proc.wait() != 0:
            failed = failed or subprocess.CalledProcessError(proc.returncode, cmd)
        else:
            os.replace(tmp, out)
    if failed:
        raise failed
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
