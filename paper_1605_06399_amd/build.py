"""Build ``libicl.so`` (HIP, gfx950) from ``csrc/`` with hipcc, in-tree.

Each source compiles to an object in ``_build/`` (in parallel), then one
``hipcc -shared`` link.  Packed-FP32 instructions are disabled for all device
code (``-packed-fp32-ops``); hipcc's host pass warns that it does not know the
feature, which is harmless.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libicl.so")

SOURCES = ["api.hip", "conv_sep.hip", "conv2d.hip", "conv2d_mfma.hip", "conv2d_u8.hip", "conv3d.hip", "harris.hip", "nms.hip", "corners.hip", "batched.hip", "bank.hip",
           "tuner.hip", "perf_model.hip"]

ARCH = os.environ.get("ICL_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(os.path.dirname(HERE), "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    noise = ("packed-fp32-ops", "warning: feature flag", "1 warning generated", "warnings generated")
    msgs = [ln for ln in (p.stdout + p.stderr).splitlines() if ln.strip() and not any(n in ln for n in noise)]
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(msgs[-60:]))
    if msgs:
        sys.stderr.write(f"[icl build] {src}:\n" + "\n".join(msgs[-20:]) + "\n")
    return obj


def build(jobs: int | None = None) -> str:
    """Compile every source and link libicl.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
