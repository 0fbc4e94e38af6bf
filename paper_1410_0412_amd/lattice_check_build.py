"""Host-only build of the lattice builder with AddressSanitizer and
UndefinedBehaviorSanitizer.

``lattice.cpp`` is plain C++ (no device code), so g++ compiles it together
with the self-check driver ``csrc/lattice_check.cpp`` into a CPU program.
The driver builds lattices of seeded masks under every periodicity and
enumeration, and the paper's empty channel, and checks every table against
its definition. Any sanitizer report aborts the program with a nonzero
status.
"""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def build(out_dir: str) -> str:
    """Compile ``lattice_check`` into ``out_dir``; returns the program's path."""
    gxx = shutil.which("g++")
    if gxx is None:
        raise RuntimeError("g++ not found")
    exe = os.path.join(out_dir, "lattice_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread"] + SAN_FLAGS + [
        "-I", INCLUDE, "-I", CSRC,
        os.path.join(CSRC, "lattice.cpp"), os.path.join(CSRC, "lattice_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("g++ failed:\n" + r.stdout + r.stderr)
    return exe


def run(exe: str, channel: bool = True, timeout: float = 600.0):
    """Run the self-check; returns the CompletedProcess."""
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return subprocess.run([exe] + (["channel"] if channel else []), capture_output=True, text=True,
                          timeout=timeout, env=env)
