"""Build the HIP library ``liblbm_sparse.so`` in-tree for gfx950.

The library holds the host lattice builder (C++) and the device solver (HIP).
It is compiled without floating-point contraction (``-ffp-contract=off``):
the FP64 collision then evaluates exactly the products and sums it spells
out, in the order it spells them out. Packed FP32 instructions are disabled.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblbm_sparse.so")

SOURCES = ["lattice.cpp", "solver.hip"]
HEADERS = ["common.hpp", "d3q19.hpp", "kernels.hpp", "adjoint.hpp"]
# the files the GPU kernels are compiled from (lattice.cpp is host code)
DEVICE_SOURCES = ["solver.hip"] + HEADERS

# the C ABI driven from C++ without Python (host code only)
DRIVER_SOURCE = "lbm_run.cpp"
DRIVER = os.path.join(HERE, "lbm_run")
DRIVER_FLAGS = ["-O2", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", INCLUDE]

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-pthread",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _run(cmd, verbose, what):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building " + what)


def build(verbose: bool = False, extra=()) -> str:
    """Compile every source into ``liblbm_sparse.so``, then the command-line
    driver ``lbm_run`` against it; returns the library's path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([hipcc()] + FLAGS + list(extra) + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp],
         verbose, "liblbm_sparse.so")
    os.replace(tmp, LIB)
    tmp = DRIVER + ".tmp%d" % os.getpid()
    _run([hipcc()] + DRIVER_FLAGS + [os.path.join(CSRC, DRIVER_SOURCE), "-L", HERE, "-llbm_sparse",
                                     "-Wl,-rpath,$ORIGIN", "-o", tmp], verbose, "lbm_run")
    os.replace(tmp, DRIVER)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
