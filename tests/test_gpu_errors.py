"""Error paths with a real device: a request above the device allocation limit fails with
Z3_ERR_OUT_OF_MEMORY and writes nothing (zeta, pair total, FFTLog output and index handle
unchanged), and the same calls succeed, with the unlimited results, once the limit is lifted;
a HIP error left pending by an earlier runtime call (an invalid device ordinal passed to the
runtime directly, which faults nothing) surfaces as Z3_ERR_HIP from the next library call
that checks the runtime, and the call after it succeeds."""

import ctypes

import numpy as np
import pytest
import torch

import paper_2408_16847_amd as z3
from paper_2408_16847_amd import _lib
from synth import CONFIGS, fftlog_inputs, make_positions, make_values
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu

OK, OOM, HIP = 0, 2, 3
SIZE_MAX = ctypes.c_size_t(-1).value


def _cap(n=3000):
    cfg = CONFIGS["cap20k"]
    xyz = make_positions(cfg, device="cuda")[:, :n].contiguous()
    x = make_values(cfg, xyz, seed=0).contiguous()
    return cfg, xyz, x


def _p(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_out_of_memory_writes_nothing():
    lib = _lib.load()
    cfg, xyz, x = _cap()
    E = cfg.edges_chord2()
    M = cfg.m_max
    idx = z3.Index(xyz, E)
    idx.set_values(x)
    ref = torch.zeros((M + 1, cfg.nbins, cfg.nbins, 2), dtype=torch.float64, device="cuda")
    pref = torch.zeros(1, dtype=torch.int64, device="cuda")
    z3.estimate_raw(idx, M, "fp64", zeta=ref, pair_total=pref)
    torch.cuda.synchronize()
    G.say("errors: oom case, pairs", int(pref.item()))
    zeta = torch.full_like(ref, 7.0)
    pairs = torch.full((1,), 12345, dtype=torch.int64, device="cuda")
    try:
        assert lib.z3_set_device_alloc_limit(ctypes.c_size_t(1 << 20)) == OK
        for prec in (0, 1):
            st = lib.z3_estimate(idx.handle, 0, M, prec, 0, idx.n, _p(zeta), _p(pairs), _stream())
            assert st == OOM and b"allocation limit" in lib.z3_last_error(), (prec, st)
        torch.cuda.synchronize()
        assert bool((zeta == 7.0).all()) and int(pairs.item()) == 12345
        # an index build under the limit (below its sorted-coordinate arrays) leaves no handle
        lib.z3_set_device_alloc_limit(ctypes.c_size_t(4096))
        out = ctypes.c_void_p()
        st = lib.z3_build_index(idx.n, _p(xyz), None, cfg.nbins, E.ctypes.data_as(ctypes.c_void_p), 0.0, _stream(),
                                ctypes.byref(out))
        assert st == OOM and out.value is None
    finally:
        lib.z3_set_device_alloc_limit(ctypes.c_size_t(SIZE_MAX))
    zeta.zero_()
    pairs.zero_()
    assert lib.z3_estimate(idx.handle, 0, M, 0, 0, idx.n, _p(zeta), _p(pairs), _stream()) == OK
    torch.cuda.synchronize()
    assert torch.equal(zeta, ref) and int(pairs.item()) == int(pref.item())
    idx.free()


def test_fftlog_out_of_memory_writes_nothing():
    lib = _lib.load()
    Pk, F, theta, _, _ = fftlog_inputs(N=64, k_max=30.0, nchi=100, nmodels=3, ntheta=12, seed=9)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Pk_d, F_d, th_d = dev(Pk), dev(F), dev(theta)
    out = torch.full((3, 3, 12, 12), 7.0, dtype=torch.float64, device="cuda")
    nu = (ctypes.c_double * 4)(-1.3, -2.5, -1.3, -1.3)
    try:
        lib.z3_set_device_alloc_limit(ctypes.c_size_t(4096))
        st = lib.z3_fftlog_a_functions(64, _p(Pk_d), 1e-6, 30.0, nu, 100, 1e-4, 60.0, 3, _p(F_d), 12, _p(th_d),
                                       _p(out), None, ctypes.c_size_t(0), _stream())
        assert st == OOM
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())
    finally:
        lib.z3_set_device_alloc_limit(ctypes.c_size_t(SIZE_MAX))
    ref = z3.fftlog_a_functions(Pk_d, 1e-6, 30.0, list(nu), F_d, 1e-4, 60.0, th_d)
    st = lib.z3_fftlog_a_functions(64, _p(Pk_d), 1e-6, 30.0, nu, 100, 1e-4, 60.0, 3, _p(F_d), 12, _p(th_d),
                                   _p(out), None, ctypes.c_size_t(0), _stream())
    torch.cuda.synchronize()
    assert st == OK and torch.equal(out, ref)


def _hip_runtime():
    """The HIP runtime this process (torch and libzeta3) already has loaded."""
    _lib.load()
    paths = [ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64" in ln]
    assert paths, "no HIP runtime mapped"
    hip = ctypes.CDLL(paths[0])
    hip.hipSetDevice.argtypes = [ctypes.c_int]
    hip.hipSetDevice.restype = ctypes.c_int
    return hip


def test_pending_runtime_error_surfaces_once():
    lib = _lib.load()
    torch.cuda.synchronize()
    assert lib.z3_sync(_stream()) == OK
    hip = _hip_runtime()
    assert hip.hipSetDevice(1 << 20) != 0  # invalid ordinal: an error code, nothing faulted
    st = lib.z3_sync(_stream())
    msg = lib.z3_last_error().decode()
    G.say("errors: pending runtime error ->", st, msg)
    assert st == HIP and msg
    assert lib.z3_sync(_stream()) == OK
    # the library keeps working
    cfg, xyz, x = _cap(1500)
    idx = z3.Index(xyz, cfg.edges_chord2())
    idx.set_values(x)
    zeta, _ = z3.estimate(idx, cfg.m_max, "fp64")
    assert np.isfinite(zeta).all()
    idx.free()
