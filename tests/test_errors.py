"""Error paths of the C ABI that need no GPU: the device allocation limit (set by call or by
Z3_DEVICE_ALLOC_LIMIT_MB) turns a too-large request into Z3_ERR_OUT_OF_MEMORY before any
device call, with no index created and the error text naming the limit; on a machine without
a GPU, calls that reach the device report Z3_ERR_HIP with the runtime's text instead of
crashing.  (The same paths under the sanitizers: tests/test_sanitizers.py; with a real
device and outputs checked for no partial writes: tests/test_gpu_errors.py.)"""

import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OK, INVALID, OOM, HIP = 0, 1, 2, 3
SIZE_MAX = ctypes.c_size_t(-1).value


def _lib():
    from paper_2408_16847_amd import _lib
    return _lib.load()


def _build(lib, n=10):
    edges = np.array([1e-6, 4e-6, 1e-5])
    out = ctypes.c_void_p()
    st = lib.z3_build_index(n, ctypes.c_void_p(0x1000), None, 2, edges.ctypes.data_as(ctypes.c_void_p), 0.0, None,
                            ctypes.byref(out))
    return st, out.value, lib.z3_last_error().decode()


def test_allocation_limit_is_out_of_memory_before_device_work():
    lib = _lib()
    try:
        assert lib.z3_set_device_alloc_limit(0) == OK
        st, handle, msg = _build(lib)
        assert st == OOM and handle is None and "allocation limit" in msg, (st, msg)
        nu = (ctypes.c_double * 4)(-1.3, -2.5, -1.3, -1.3)
        fake = ctypes.c_void_p(0x1000)
        st = lib.z3_fftlog_a_functions(64, fake, 1e-6, 30.0, nu, 100, 1e-4, 60.0, 2, fake, 8, fake, fake, None,
                                       ctypes.c_size_t(0), None)
        assert st == OOM and "allocation limit" in lib.z3_last_error().decode()
        # argument errors still take precedence over the limit
        st = lib.z3_fftlog_a_functions(63, fake, 1e-6, 30.0, nu, 100, 1e-4, 60.0, 2, fake, 8, fake, fake, None,
                                       ctypes.c_size_t(0), None)
        assert st == INVALID
    finally:
        lib.z3_set_device_alloc_limit(ctypes.c_size_t(SIZE_MAX))


def test_allocation_limit_from_the_environment():
    code = ("import ctypes, numpy as np\n"
            "from paper_2408_16847_amd import _lib\n"
            "lib = _lib.load()\n"
            "e = np.array([1e-6, 4e-6, 1e-5]); out = ctypes.c_void_p()\n"
            "st = lib.z3_build_index(10, ctypes.c_void_p(0x1000), None, 2, e.ctypes.data_as(ctypes.c_void_p), 0.0,"
            " None, ctypes.byref(out))\n"
            "print(st, out.value, lib.z3_last_error().decode())\n")
    env = dict(os.environ, Z3_DEVICE_ALLOC_LIMIT_MB="0")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    st, handle, msg = r.stdout.strip().split(" ", 2)
    assert int(st) == OOM and handle == "None" and "allocation limit" in msg


def test_without_a_device_calls_report_hip_errors():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib()
    st = lib.z3_sync(None)
    assert st == HIP and lib.z3_last_error().decode().startswith("hipStreamSynchronize")
    st, handle, msg = _build(lib)
    assert st == HIP and handle is None and msg
