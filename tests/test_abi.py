"""C ABI checks that need no GPU: the library loads, exports every declared symbol, and
rejects invalid arguments on the host side before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zeta3.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(z3_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("z3_build_index", "z3_accumulate_multipoles", "z3_contract", "z3_estimate", "z3_resum",
              "z3_finalize", "z3_index_free"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2408_16847_amd import _lib
    lib = _lib.load()
    for s in declared_symbols():
        assert hasattr(lib, s), s
        assert s in _lib.SIGNATURES, s


def test_no_other_exported_symbols():
    import subprocess
    from paper_2408_16847_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    z3 = {s for s in exported if s.startswith("z3_")}
    assert z3 == set(declared_symbols())


def _edges():
    return np.array([1e-6, 4e-6, 1e-5])


def _status(name, *args):
    from paper_2408_16847_amd import _lib
    lib = _lib.load()
    return getattr(lib, name)(*args), lib.z3_last_error().decode()


def test_build_index_rejects_bad_arguments_without_a_device():
    P = ctypes.c_void_p
    out = ctypes.c_void_p()
    good = _edges()
    cases = [
        (-1, good, 2, "n < 0"),
        (10, np.array([0.0, 1e-5, 2e-5]), 2, "E_0"),
        (10, np.array([1e-5, 1e-5, 2e-5]), 2, "strictly increasing"),
        (10, np.array([1e-5, 2e-5, 5.0]), 2, "E_nbins > 4"),
        (10, np.array([1e-5, np.nan, 2e-5]), 2, "not finite"),
        (10, good, 0, "nbins"),
        (10, good, 65, "nbins"),
    ]
    for n, e, nb, msg in cases:
        e = np.ascontiguousarray(e)
        st, err = _status("z3_build_index", n, P(1), P(0), nb, e.ctypes.data_as(P), 0.0, P(0), ctypes.byref(out))
        assert st == 1, (msg, st, err)
        assert msg in err, (msg, err)
        assert out.value is None
    st, err = _status("z3_build_index", 10, P(0), P(0), 2, good.ctypes.data_as(P), 0.0, P(0), ctypes.byref(out))
    assert st == 1 and "xyz" in err
    st, err = _status("z3_build_index", 1 << 31, P(1), P(0), 2, good.ctypes.data_as(P), 0.0, P(0), ctypes.byref(out))
    assert st == 5


def test_other_entry_points_reject_bad_arguments():
    P = ctypes.c_void_p
    assert _status("z3_accumulate_multipoles", P(0), 0, 4, 0, 0, 0, 1, P(0), P(0), P(0), P(0), P(0), P(0))[0] == 1
    assert _status("z3_estimate", P(0), 0, 4, 0, 0, 1, P(1), P(0), P(0))[0] == 1
    assert _status("z3_estimate_ex", P(0), 0, 4, 0, 1, 0, 1, P(1), P(0), P(0))[0] == 1
    assert _status("z3_estimate_static", P(0), 0, 4, 0, 0, 0, 1, P(1), P(0), P(0))[0] == 1
    assert _status("z3_index_set_phi_bins", P(0), 16, P(1))[0] == 1
    assert _status("z3_accumulate_histogram", P(0), 0, 4, 0, 0, 0, 1, P(0), P(0), P(0), P(0), P(0), P(0))[0] == 1
    assert _status("z3_estimate_histogram", P(0), 0, 4, 0, 0, 1, P(1), P(0), P(0))[0] == 1
    assert _status("z3_estimate_cross", P(0), 0, 1, 2, 1, 4, 0, 0, 1, P(1), P(0), P(0))[0] == 1
    assert _status("z3_estimate_cross_catalogues", P(0), 0, P(0), 0, 1, P(1), P(0), P(1), 4, 0, 0, 1, P(1),
                   P(0), P(0), P(0), P(0))[0] == 1
    out = P()
    good = np.array([1.0, 4.0])
    assert _status("z3_build_index_planar", 1, P(0), P(0), 1, good.ctypes.data_as(P), 0.0, P(0),
                   ctypes.byref(out))[0] == 1
    bad = np.array([0.0, 4.0])
    assert _status("z3_build_index_planar", 1, P(1), P(0), 1, bad.ctypes.data_as(P), 0.0, P(0),
                   ctypes.byref(out))[0] == 1
    assert _status("z3_contract", 10, 128, 4, 0, P(1), P(1), P(1), P(0))[0] == 1
    assert _status("z3_contract", 10, 4, 4, 7, P(1), P(1), P(1), P(0))[0] == 1
    assert _status("z3_contract", 10, 4, 4, 0, P(1), P(1), P(0), P(0))[0] == 1
    assert _status("z3_resum", 4, 65, P(1), 3, P(1), P(1), P(0))[0] == 1
    assert _status("z3_resum", 128, 4, P(1), 3, P(1), P(1), P(0))[0] == 1
    assert _status("z3_finalize", 1, 128, 4, P(1), P(1), P(0))[0] == 1
    assert _status("z3_finalize", 0, 4, 4, P(1), P(1), P(0))[0] == 1
    assert _status("z3_index_info", P(0), P(0), P(0), P(0), P(0), P(0))[0] == 1
    # index-based calls with a NULL index
    assert _status("z3_estimate_maps", P(0), 4, 0, 0, 1, P(1), P(0), P(0))[0] == 1
    assert _status("z3_estimate_pivots", P(0), 0, 1, P(1), P(0), P(1), 4, 0, 0, 1, P(1), P(0), P(0), P(0))[0] == 1
    assert _status("z3_adjoint", P(0), 0, 4, 0, 1, P(1), 1.0, P(1), P(0))[0] == 1
    assert _status("z3_adjoint_maps", P(0), 4, 0, 1, P(1), 1.0, P(1), P(0))[0] == 1
    assert _status("z3_pivot_weight_sum", P(0), 0, 1, P(1), P(0))[0] == 1
    assert _status("z3_index_update_values", P(0), P(1), P(0))[0] == 1
    assert _status("z3_index_prepare_capture", P(0), 0, P(0))[0] == 1
    assert _status("z3_index_set_batch_shape", P(0), 0, 0)[0] == 1
    assert _status("z3_index_batch_shape", P(0), 10, 0, P(1), P(1))[0] == 1
    # empty work is a successful no-op
    assert _status("z3_contract", 0, 4, 4, 0, P(0), P(0), P(1), P(0))[0] == 0
    assert _status("z3_resum", 4, 4, P(0), 0, P(0), P(0), P(0))[0] == 0


def test_status_strings():
    from paper_2408_16847_amd import _lib
    lib = _lib.load()
    names = [lib.z3_status_string(i).decode() for i in range(6)]
    assert names[0] == "ok" and len(set(names)) == 6
