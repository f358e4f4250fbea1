"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer: its pins (the
brute-force equality, closed forms, invariants, the iMBEA variant's pins) run in a child
process against a sanitized build, so that an out-of-bounds access, a use after free, a
signed overflow or a misaligned load in the oracle aborts the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_sanitizers():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc's sanitizer runtimes are not installed")
    env = dict(os.environ, MBE_ORACLE_SANITIZE="1", LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("PYTEST_ADDOPTS", None)
    cmd = [sys.executable, "-c",
           "import oracle; oracle.build(force=True)"]
    subprocess.run(cmd, cwd=ROOT, env=env, check=True, timeout=300)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle.py", "tests/test_oracle_pins.py", "tests/test_oracle_imbea.py",
                        "tests/test_oracle_pivot.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
