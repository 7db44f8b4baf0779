"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU oracle tests
(pins, planted-mistake checks excluded: they compile their own copies) run again in a child process
that loads the instrumented build with the ASan runtime preloaded; any finding aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    try:
        path = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _env():
    asan = _runtime()
    if asan is None or os.environ.get("LD_PRELOAD"):
        pytest.skip("gcc's ASan runtime is not available here (or a preload is already set)")
    import oracle
    oracle.build(sanitize=True)
    return dict(os.environ, OPMM_ORACLE_SANITIZE="1", LD_PRELOAD=asan,
                ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")


PLANTED = """
import re, numpy as np, oracle
L = oracle.lib()
maps = open('/proc/self/maps').read()
assert 'libopmm_oracle_san.so' in maps and 'libasan' in maps, 'instrumented build not loaded'
print('loaded', flush=True)
short = np.zeros(4)                       # the call writes 18 values: a planted overflow
L.oracle_nominal(43.0, short.ctypes.data)
print('not caught', flush=True)
"""


@pytest.mark.slow
def test_sanitized_build_is_loaded_and_catches_an_overflow():
    """The child loads the instrumented build, and a call handed a too-short output buffer is stopped
    with a heap-buffer-overflow report."""
    r = subprocess.run([sys.executable, "-c", PLANTED], cwd=ROOT, env=_env(), capture_output=True,
                       text=True, timeout=300)
    assert "loaded" in r.stdout, r.stdout + r.stderr[-2000:]
    assert r.returncode != 0 and "not caught" not in r.stdout
    assert "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]


@pytest.mark.slow
def test_oracle_tests_pass_under_sanitizers():
    env = _env()
    files = [os.path.join(ROOT, "tests", f) for f in ("test_oracle.py", "test_ivt.py", "test_polish.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *files], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail
