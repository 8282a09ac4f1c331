"""Compile the HIP library libpwfs.so in-tree for gfx950 (hipcc, no JIT)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libpwfs.so")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("pwfs_kernels.hip", "pwfs_kernels16.hip",
                                                  "pwfs_detector.hip", "pwfs_psf.hip", "pwfs_sh.hip", "pwfs_fstop.hip", "pwfs_static.hip",
                                                  "pwfs_api.cpp",
                                                  "cnn_kernels.hip", "cnn_api.cpp")]
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # Packed FP32 VALU forms stay disabled for all device code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), *FLAGS, *(extra or []), "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
