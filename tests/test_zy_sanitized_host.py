"""The host code of the rasterizer library and the FP64 oracle under
AddressSanitizer and UndefinedBehaviorSanitizer.

Both are rebuilt with the sanitizers (the library's host code only: every
flag is behind -Xarch_host, the gfx950 device code is built as always), and
the CPU tests that load them -- argument validation of every entry point,
the host side of the partitioning, the oracle's pins -- run again in a child
process with clang's runtime preloaded.  Any sanitizer report fails the
test.  The central-difference check at the 200k-Gaussian scale is left out:
without OpenMP under the sanitizers it alone takes minutes.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ["tests/test_abi.py", "tests/test_partition.py", "tests/test_oracle.py", "tests/test_oracle_adam.py",
         "tests/test_oracle_appearance.py", "tests/test_oracle_loss.py", "tests/test_oracle_partition.py"]

CHECK_LOADED = """
import paper_2402_17427_amd._native as N, oracle
N.lib(); oracle.lib()
maps = open('/proc/self/maps').read()
for name in ('libclang_rt.asan', 'libgsmi_san.so', 'liboracle_san.so'):
    assert name in maps, name
print('sanitized builds loaded')
"""


def test_cpu_side_under_address_and_undefined_behaviour_sanitizers():
    if os.environ.get("GS_UNDER_SANITIZERS"):
        pytest.skip("already inside the sanitized run")
    sys.path.insert(0, ROOT)
    import oracle
    from paper_2402_17427_amd import build as b
    env = dict(os.environ,
               LD_PRELOAD=b.sanitizer_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               GSMI_LIB=b.build(sanitize=True),
               GS_ORACLE_LIB=oracle.build_sanitized(),
               GS_UNDER_SANITIZERS="1")
    r = subprocess.run([sys.executable, "-c", CHECK_LOADED], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "sanitized builds loaded" in r.stdout, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        "-k", "not c3_scale"] + FILES, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert " passed" in out
