"""Builds the gfx950 shared library liblbm.so in this directory with hipcc."""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["lbm_kernels.hip", "lbm_api.hip", "nn_kernels.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result",
    # The small-tile 16-bit instances are limited to three blocks per CU by
    # their LDS, below the four waves per SIMD the register budget aims at.
    "-Wno-pass-failed",
    # Fuse a * b + c only within one source expression: the fusion choices
    # are then the same in every instantiation of the step (each mode, tile
    # and the batched form), so they all produce the same bits.
    "-ffp-contract=on",
]


def source_digest() -> str:
    """Digest of the step kernel source and of the host code that lays out
    its data and chooses its launch (what a traffic profile or a launch-shape
    timing depends on), over their code lines only: '//' comments and blank
    lines are left out.  16 hex digits."""
    h = hashlib.sha256()
    for name in ("lbm_kernels.hip", "lbm_api.hip"):
        with open(os.path.join(CSRC, name), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs, procs = [], []
    for src in SOURCES:   # the translation units compile in parallel
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for proc, cmd in procs:
        if proc.wait() != 0:
            raise subprocess.CalledProcessError(proc.returncode, cmd)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
