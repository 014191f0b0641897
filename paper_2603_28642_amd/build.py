"""Build the HIP library librsilu.so for gfx950, in tree.

The host setup (setup.cpp) is compiled by g++ with -ffp-contract=off so the
factorization's floating-point decisions are reproducible; the kernels, the
C ABI, the batched persistent solves (*.hip) and the serving runtime (serve.cpp)
by hipcc for gfx950.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "librsilu.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
INCLUDES = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _run(cmd, quiet):
    if not quiet:
        print(" ".join(cmd), file=sys.stderr, flush=True)
    subprocess.run(cmd, check=True)


def build(quiet=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    setup_o = os.path.join(OUT_DIR, "setup.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
          "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include")] + INCLUDES +
         ["-c", os.path.join(CSRC, "setup.cpp"), "-o", setup_o], quiet)
    objs.append(setup_o)
    for name in ("kernels.hip", "capi.hip", "batch.hip", "serve.cpp"):
        o = os.path.join(OUT_DIR, name.rsplit(".", 1)[0] + ".o")
        _run([HIPCC] + HIP_FLAGS + INCLUDES + ["-c", os.path.join(CSRC, name), "-o", o], quiet)
        objs.append(o)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs, quiet)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
