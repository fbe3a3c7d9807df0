"""Build libtc3d.so (the HIP library behind include/tc3d.h) in-tree for gfx950.

    python -m paper_2212_06985_amd.build
"""
from __future__ import annotations

import glob
import hashlib
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtc3d.so")

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # packed FP32 instructions stay off: the compiler must not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


def source_files() -> list:
    """Every file the library is built from, in a fixed order."""
    return (sorted(glob.glob(os.path.join(CSRC, "*.hip"))) +
            sorted(glob.glob(os.path.join(CSRC, "*.hpp"))) +
            [os.path.join(ROOT, "include", "tc3d.h")])


def source_id() -> str:
    """SHA-256 over the sources' names and contents; the library returns the
    value it was built with from tc3d_build_id()."""
    h = hashlib.sha256()
    for f in source_files():
        h.update(os.path.relpath(f, ROOT).encode())
        h.update(b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, f'-DTC3D_BUILD_ID="{source_id()}"', "-I",
           os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 feature and says so; that
    # note is expected, anything else is shown
    noise = "'-packed-fp32-ops' is not a recognized feature"
    other = [ln for ln in res.stderr.splitlines() if noise not in ln and ln.strip()]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(other))
    if other and verbose:
        print("\n".join(other), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
