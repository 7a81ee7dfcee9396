"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds oracle/libldu_oracle_san.so (gcc -fsanitize=address,undefined,
-fno-sanitize-recover=all) and runs the oracle's pins and golden checks in a
child process that preloads the ASan runtime: any out-of-bounds access,
use-after-free or undefined behaviour in the oracle aborts the child and
fails this test.  Leak checking is off (the Python interpreter itself holds
allocations at exit).  CPU only.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                           text=True, timeout=30)
    except (OSError, subprocess.TimeoutExpired):
        return None
    path = p.stdout.strip()
    return path if p.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(_asan_runtime() is None, reason="gcc's ASan runtime is not installed")
def test_oracle_pins_pass_under_asan_and_ubsan():
    env = dict(os.environ)
    env.update(ORACLE_SANITIZE="1", LD_PRELOAD=_asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    sys.path.insert(0, ROOT)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"),
           os.path.join(ROOT, "tests", "test_oracle_golden.py")]
    p = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    err = p.stderr
    k = max(err.find("ERROR: AddressSanitizer"), err.find("runtime error"))
    report = err[k:k + 3000] if k >= 0 else ""
    tail = report + (p.stdout + p.stderr)[-2000:]
    assert p.returncode == 0, tail
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, tail
    assert os.path.exists(os.path.join(ROOT, "oracle", "libldu_oracle_san.so"))
