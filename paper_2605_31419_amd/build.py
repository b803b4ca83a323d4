"""Build of the gfx950 HIP library (``libtsr.so``) from ``csrc/``.

hipcc cross-compiles for gfx950 without a GPU.  Packed-FP32 instruction selection is
disabled (-packed-fp32-ops); float atomics are the hardware ones (coarse-grained memory).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtsr.so")

SOURCES = ["tsr_bin.hip", "tsr_blend.hip", "tsr_ssim.hip", "tsr_reg.hip", "tsr_normal.hip", "tsr_api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-fvisibility=hidden",
    "-Wall", "-Wno-unused-function",
]


def source_fingerprint() -> str:
    """SHA-256 over the kernel sources, the public header and the compiler flags: profiler
    counters recorded under one fingerprint describe exactly that build."""
    import hashlib

    h = hashlib.sha256(" ".join(FLAGS).encode())
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".h")))
    for f in files + ["../../include/tsr.h"]:
        with open(os.path.normpath(os.path.join(CSRC, f)), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()


def build(verbose: bool = False, extra=None, out: str = LIB) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *(extra or []), "-I", INCLUDE, "-I", CSRC, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
