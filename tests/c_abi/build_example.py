"""Build the C ABI example (tests/c_abi/dsmc_c_example.cpp) against the
in-tree library: hipcc for the host code only, linked to
paper_2301_05985_amd/_lib/libdsmc_hip.so with a relative run path."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
SRC = os.path.join(HERE, "dsmc_c_example.cpp")
OUT = os.path.join(HERE, "_build", "dsmc_c_example")


def build():
    from paper_2301_05985_amd import build as B
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    libdir = os.path.dirname(B.LIB)
    rel = os.path.relpath(libdir, os.path.dirname(OUT))
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call([B.hipcc(), "-O2", "-std=c++17", "-Wall", SRC, "-o", tmp, "-L", libdir, "-ldsmc_hip",
                           "-Wl,-rpath,$ORIGIN/" + rel])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
