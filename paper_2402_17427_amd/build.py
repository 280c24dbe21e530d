"""Build the HIP rasterizer library (gfx950) in-tree.

`build()` compiles every source under csrc/ with hipcc into
`libgsmi.so` next to this file.  Packed FP32 instructions are disabled
(`-packed-fp32-ops` off) and FP contraction is left to the explicit fmaf
calls in the kernels, so that the forward and backward blend take
bit-identical decisions.
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsmi.so")
ARCH = os.environ.get("GSMI_ARCH", "gfx950")

SOURCES = ["api.cpp", "profile.cpp", "project.hip", "binning.hip", "sort.hip", "render_fwd.hip", "render_bwd.hip",
           "batch_kernels.hip", "loss.hip", "optim.hip", "partition.hip", "partition.cpp", "appearance.hip", "appearance.cpp", "batch.cpp", "serve.cpp"]
EXTRA_SOURCES = []


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    out = [os.path.join(CSRC, s) for s in SOURCES]
    out += [os.path.join(CSRC, s) for s in EXTRA_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    return out


def build(verbose: bool = False, defines=(), out: str | None = None) -> str:
    """Compile the library; `defines` are extra -D options (tuning
    constants), `out` another output path (default libgsmi.so here)."""
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-munsafe-fp-atomics",
           # atomics are issued from one lane where it matters; the
           # compiler's lane-loop rewrite of uniform-address atomics only
           # adds instructions there
           "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
           "-I", os.path.join(HERE, "..", "include"), "-o", tmp] + [f"-D{d}" for d in defines] + sources() + ["-lpthread"]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
