"""The C-ABI library's host code under AddressSanitizer + UndefinedBehaviorSanitizer (the device code
is built as in the product library): the ABI tests -- symbol table, struct layouts, host-only calls,
null handles, context creation failing cleanly without a GPU -- run again in a child process that
loads the host-instrumented build with clang's ASan runtime preloaded.  A planted overflow (a host
call handed a too-short output buffer) must be caught."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _env():
    from paper_2007_09884_amd import build as B
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("a preload is already set")
    if not os.path.exists(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc is not available")
    lib = B.san_lib("address,undefined")
    if not os.path.exists(lib) or any(os.path.getmtime(d) > os.path.getmtime(lib) for d in B.DEPS):
        B.build(sanitize="address,undefined")
    rt = B.sanitizer_runtime("asan")
    if not os.path.exists(rt):
        pytest.skip("clang's ASan runtime is not available")
    return dict(os.environ, OPMM_LIBRARY=lib, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0",
                UBSAN_OPTIONS="print_stacktrace=1")


PLANTED = """
import numpy as np
from paper_2007_09884_amd import opmm
maps = open('/proc/self/maps').read()
assert 'libopmm_host_asan.so' in maps and 'clang_rt.asan' in maps, 'instrumented build not loaded'
print('loaded', flush=True)
short = np.zeros(4, np.float32)             # opmm_nominal writes 18 values: a planted overflow
opmm.lib.opmm_nominal(43.0, short.ctypes.data)
print('not caught', flush=True)
"""


@pytest.mark.slow
def test_host_build_catches_a_planted_overflow():
    r = subprocess.run([sys.executable, "-c", PLANTED], cwd=ROOT, env=_env(), capture_output=True,
                       text=True, timeout=600)
    assert "loaded" in r.stdout, r.stdout + r.stderr[-2000:]
    assert r.returncode != 0 and "not caught" not in r.stdout
    assert "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]


@pytest.mark.slow
def test_abi_tests_pass_on_the_host_sanitized_build():
    env = _env()
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail
