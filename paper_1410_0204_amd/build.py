"""Builds libtmm.so (HIP, gfx950) in-tree next to this file."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtmm.so")
SOURCES = [os.path.join(HERE, "csrc", "tmm.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("tmm_device.hpp", "tmm_persistent.hpp", "tmm_substep.hpp",
                                                   "tmm_probe.hpp")] + [
    os.path.join(ROOT, "include", "tmm.h")]


def source_hash():
    """Hash of the HIP sources the library is built from (keys measured kernel data to a build)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("tmm_device.hpp", "tmm_persistent.hpp", "tmm_substep.hpp", "tmm_probe.hpp", "tmm.hip"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def command(out):
    return [
        "hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-Wall", "-Wno-unused-result",
        # packed float32 instructions stay disabled for all device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
        "-o", out, *SOURCES,
    ]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
