"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):

* the C oracle (oracle/oracle_cpu.c) with gcc's sanitizers, driven by
  tests/sanitize/oracle_checks.c on a small seeded catalogue;
* the host side of libzeta3 (argument validation, status codes, error text, the allocation
  limit, the FFTLog entry's checks), built with -fsanitize on the host pass only and driven by
  tests/sanitize/abi_checks.c, whose calls all end before any device work.

The instrumented library is built once per source state under _build/ (about a minute)."""

import hashlib
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(ROOT, "_build", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_asan_ubsan():
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_checks")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", os.path.join(ROOT, "oracle", "oracle_cpu.c"),
          os.path.join(SAN, "oracle_checks.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV)
    assert "oracle checks ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def _sanitized_library():
    from paper_2408_16847_amd import build
    srcs = sorted(glob.glob(os.path.join(build.SRC_DIR, "*"))) + [os.path.join(ROOT, "include", "zeta3.h")]
    h = hashlib.sha256(" ".join(HOST_SAN).encode())
    for f in srcs:
        h.update(open(f, "rb").read())
    lib = os.path.join(OUT, "libzeta3_san.so")
    stamp = lib + ".sha256"
    if os.path.exists(lib) and os.path.exists(stamp) and open(stamp).read() == h.hexdigest():
        return lib
    os.makedirs(OUT, exist_ok=True)
    build.build(lib=lib, extra=HOST_SAN, jobs=8)
    open(stamp, "w").write(h.hexdigest())
    return lib


def test_abi_validation_under_asan_ubsan():
    if not (os.path.exists(CLANG) and shutil.which("/opt/rocm/bin/hipcc")):
        pytest.skip("ROCm clang / hipcc not available")
    lib = _sanitized_library()
    exe = os.path.join(OUT, "abi_checks")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          "-I", os.path.join(ROOT, "include"), os.path.join(SAN, "abi_checks.c"), lib,
          f"-Wl,-rpath,{os.path.dirname(lib)}", "-o", exe])
    r = _run([exe], env=ENV)
    assert "abi checks ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
