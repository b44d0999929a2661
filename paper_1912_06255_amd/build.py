"""Compile the HIP library (gfx950) into the package directory.

    python -m paper_1912_06255_amd.build

The library is built in-tree so that it travels with the source tree; nothing is
installed.  Flags:
  -ffp-contract=off    the float64 distance decision must not fuse multiply-adds;
  -packed-fp32-ops off packed FP32 instructions are not emitted.
"""

from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "dbscan.hip")
LIB = os.path.join(HERE, "libdbscan_hip.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, out: str | None = None, defines: tuple = ()) -> str:
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, *[f"-D{d}" for d in defines], "-o", tmp, SRC]
    t0 = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed ({res.returncode})")
    if verbose:
        noise = "not a recognized feature for this target"
        for line in (res.stdout + res.stderr).splitlines():
            if noise not in line:
                sys.stderr.write(line + "\n")
        print(f"built {lib} in {time.time() - t0:.1f}s")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
