"""Builds the reference CPU implementation.

* ``liboracle.so`` -- the build the tests check against: plain gcc, no
  architecture-specific flags (it is built on one machine and may run on
  another), single-threaded.
* ``build_timing(out)`` -- the CPU-baseline build of the same source:
  ``-O3 -march=native -fopenmp`` with floating-point contraction off, built
  on the machine that runs it.  Each output element is computed in the same
  order as in the plain build, so the results are the same bit for bit.
* ``build_sanitized(out)`` -- the same source with AddressSanitizer and
  UndefinedBehaviorSanitizer, linked with ``sanitize_main.c`` into a
  stand-alone program (a sanitizer runtime cannot be loaded into a running
  Python), which runs the oracle's entry points on inputs from a file.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "tmm_oracle.c")
COMMON = ["-std=c11", "-fno-fast-math", "-Wall", "-Wextra"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    _run(["gcc", "-O2", "-fPIC", "-shared", *COMMON, "-o", tmp, SRC, "-lm"], verbose)
    os.replace(tmp, LIB)
    return LIB


def build_timing(out: str, verbose: bool = False) -> str:
    tmp = out + ".tmp"
    _run(["gcc", "-O3", "-march=native", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", *COMMON,
          "-o", tmp, SRC, "-lm"], verbose)
    os.replace(tmp, out)
    return out


def build_sanitized(out: str, verbose: bool = False) -> str:
    tmp = out + ".tmp"
    _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", *COMMON, "-o", tmp, SRC, os.path.join(HERE, "sanitize_main.c"), "-lm"],
         verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
