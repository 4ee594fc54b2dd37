"""Build librmc.so (the HIP/gfx950 library behind include/mcrad.h) in-tree.

    python -m paper_1608_05238_amd.build

Always recompiles.  Flags: gfx950 only; hardware FP atomics
(-munsafe-fp-atomics); packed FP32 instructions disabled for the device.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRCS = [os.path.join(PKG, "csrc", n) for n in ("mcrad.hip", "denoise.hip", "microbench.hip")]
OUT = os.path.join(PKG, "librmc.so")
INCLUDE = os.path.join(ROOT, "include")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags() -> list:
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-munsafe-fp-atomics",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + INCLUDE]


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp"
    cmd = [hipcc()] + flags() + SRCS + ["-o", tmp]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building librmc.so")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} in {time.time() - t0:.1f}s")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
