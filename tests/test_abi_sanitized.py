"""The library's host code (argument checks, CSR validation on the host, batch packing and its
64-bit size checks) under AddressSanitizer and UndefinedBehaviorSanitizer: mbe_api.hip is
compiled with the sanitizers on its host side only, linked with the other objects of the
build, and the C-ABI tests (tests/test_abi.py, no device work) run against that copy in a
child process."""
import glob
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2401_05039_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_host_code_under_sanitizers():
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    objs = [os.path.join(PKG, "_build", f) for f in ("mbe_search.o", "mbe_prep.o", "mbe_records.o")]
    if not rt or not os.path.exists(HIPCC) or not all(os.path.exists(o) for o in objs):
        pytest.skip("hipcc, the clang sanitizer runtime or the library's objects are missing (build first)")
    d = tempfile.mkdtemp(prefix="mbe_san_")
    api = os.path.join(d, "mbe_api.o")
    so = os.path.join(d, "libmbe_san.so")
    subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), "-c", os.path.join(PKG, "csrc", "mbe_api.hip"), "-o", api],
                   check=True, capture_output=True, timeout=600)
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", so, api, *objs],
                   check=True, capture_output=True, timeout=300)
    env = dict(os.environ, MBE_LIB=so, LD_PRELOAD=rt[-1],
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_abi.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
