"""Build the HIP rasterizer library (gfx950) in-tree.

`build()` compiles every source under csrc/ with hipcc, one process per
source in parallel (objects under _build/), and links `libgsmi.so` next to
this file.  Packed FP32 instructions are disabled (`-packed-fp32-ops` off)
and FP contraction is left to the explicit fmaf calls in the kernels, so
that the forward and backward blend take bit-identical decisions.

`build(sanitize=True)` builds `libgsmi_san.so`: the same library with
AddressSanitizer and UndefinedBehaviorSanitizer on the host code only
(every flag behind -Xarch_host; the device code is compiled as always).
The sanitizer runtime is not linked in: the process that loads the library
must preload clang's ASan runtime (`sanitizer_runtime()`), and runs the CPU
side only (argument validation, the host partitioning, the server's
admission logic).
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsmi.so")
LIB_SAN = os.path.join(HERE, "libgsmi_san.so")
ARCH = os.environ.get("GSMI_ARCH", "gfx950")

SOURCES = ["api.cpp", "profile.cpp", "project.hip", "binning.hip", "sort.hip", "bin_direct.hip", "render_fwd.hip", "render_bwd.hip",
           "batch_kernels.hip", "loss.hip", "optim.hip", "partition.hip", "partition.cpp", "appearance.hip", "appearance.cpp", "batch.cpp", "serve.cpp"]
EXTRA_SOURCES = []

SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sanitizer_runtime() -> str:
    """clang's shared ASan runtime (it carries the UBSan handlers too)."""
    root = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "llvm", "lib", "clang")
    for ver in sorted(os.listdir(root), reverse=True) if os.path.isdir(root) else []:
        for rel in ("lib/linux/libclang_rt.asan-x86_64.so", "lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so"):
            p = os.path.join(root, ver, rel)
            if os.path.exists(p):
                return p
    raise RuntimeError("clang ASan runtime not found")


def sources():
    out = [os.path.join(CSRC, s) for s in SOURCES]
    out += [os.path.join(CSRC, s) for s in EXTRA_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    return out


def _flags(defines, sanitize):
    return ([f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             "-ffp-contract=off", "-munsafe-fp-atomics",
             # atomics are issued from one lane where it matters; the
             # compiler's lane-loop rewrite of uniform-address atomics only
             # adds instructions there
             "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
             "-I", os.path.join(HERE, "..", "include")] + [f"-D{d}" for d in defines] +
            (SANITIZE_FLAGS if sanitize else []))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def build(verbose: bool = False, defines=(), out: str | None = None, sanitize: bool = False,
          jobs: int | None = None) -> str:
    """Compile the library; `defines` are extra -D options (tuning
    constants), `out` another output path (default libgsmi.so here, or
    libgsmi_san.so with `sanitize`), `jobs` parallel compiles (default: the
    CPUs, at most 8)."""
    lib = out or (LIB_SAN if sanitize else LIB)
    tag = os.path.splitext(os.path.basename(lib))[0]
    objdir = os.path.join(HERE, "_build", tag)
    os.makedirs(objdir, exist_ok=True)
    flags = _flags(defines, sanitize)
    srcs = sources()
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    n = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max(1, n)) as ex:
        list(ex.map(lambda so: _run([hipcc()] + flags + ["-c", so[0], "-o", so[1]], verbose), zip(srcs, objs)))
    tmp = lib + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", "-fPIC", "-shared", "-o", tmp] + objs + ["-lpthread"], verbose)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    import sys
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
