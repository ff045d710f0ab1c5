"""ctypes wrapper of the compiled C oracle (oracle_cpu.c) -- test infrastructure only."""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build
from . import ref

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.zo_multipoles.argtypes = [I64, P, P, P, P, P, I64, P, P, P, ctypes.c_int, P, ctypes.c_int,
                                      P, P, P, P, P, P, ctypes.c_int]
        lib.zo_multipoles.restype = ctypes.c_int
        lib.zo_zeta.argtypes = [I64, P, P, P, P, P, I64, P, P, P, P, P, ctypes.c_int, P, ctypes.c_int,
                                P, P, ctypes.c_int]
        lib.zo_zeta.restype = ctypes.c_int
        lib.zo_setup_seconds.argtypes = [I64, P, P, P, P, P, ctypes.c_int, P, ctypes.c_int]
        lib.zo_setup_seconds.restype = ctypes.c_double
        _lib = lib
    return _lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def multipoles(piv, nbr, w, x, edges, m_max, ids=False, nthreads=0):
    """Per-pivot raw multipoles (a complex [P, m_max+1, nb], W [P, nb], N [P, nb]);
    with ids=True also the per-bin sum of neighbour indices and of mix64(index)."""
    lib = _load()
    nbr = _c(nbr)
    piv = _c(piv)
    w = _c(w)
    v = _c(np.asarray(w, np.float64) * np.asarray(x, np.float64))
    edges = _c(edges)
    n, P, nb = nbr.shape[1], piv.shape[1], len(edges) - 1
    nx, ny, nz = _c(nbr[0]), _c(nbr[1]), _c(nbr[2])
    px, py, pz = _c(piv[0]), _c(piv[1]), _c(piv[2])
    ar = np.zeros((P, m_max + 1, nb))
    ai = np.zeros((P, m_max + 1, nb))
    W = np.zeros((P, nb))
    N = np.zeros((P, nb), dtype=np.int64)
    isum = np.zeros((P, nb), dtype=np.uint64) if ids else None
    ihash = np.zeros((P, nb), dtype=np.uint64) if ids else None
    rc = lib.zo_multipoles(n, _ptr(nx), _ptr(ny), _ptr(nz), _ptr(w), _ptr(v), P, _ptr(px), _ptr(py), _ptr(pz),
                           nb, _ptr(edges), m_max, _ptr(ar), _ptr(ai), _ptr(W), _ptr(N),
                           _ptr(isum), _ptr(ihash), nthreads)
    if rc:
        raise RuntimeError("zo_multipoles failed")
    a = ar + 1j * ai
    if ids:
        return a, W, N, isum, ihash
    return a, W, N


def estimate(piv, nbr, w, x, edges, m_max, wp, xp, nthreads=0, self_pairs=True):
    """zeta [m_max+1, nb, nb] complex (normalised by sum w_p) and the pair total.

    self_pairs=False removes the k = j terms of the diagonal (ref.self_pair_term), with
    Q_{p,b} taken as the m = 0 multipole of the field w x^2.
    """
    lib = _load()
    nbr = _c(nbr)
    piv = _c(piv)
    w = _c(w)
    v = _c(np.asarray(w, np.float64) * np.asarray(x, np.float64))
    wp = _c(wp)
    pv = _c(np.asarray(wp, np.float64) * np.asarray(xp, np.float64))
    edges = _c(edges)
    n, P, nb = nbr.shape[1], piv.shape[1], len(edges) - 1
    nx, ny, nz = _c(nbr[0]), _c(nbr[1]), _c(nbr[2])
    px, py, pz = _c(piv[0]), _c(piv[1]), _c(piv[2])
    zeta = np.zeros((m_max + 1, nb, nb, 2))
    pairs = np.zeros(1, dtype=np.int64)
    rc = lib.zo_zeta(n, _ptr(nx), _ptr(ny), _ptr(nz), _ptr(w), _ptr(v), P, _ptr(px), _ptr(py), _ptr(pz),
                     _ptr(wp), _ptr(pv), nb, _ptr(edges), m_max, _ptr(zeta), _ptr(pairs), nthreads)
    if rc:
        raise RuntimeError("zo_zeta failed")
    z = zeta[..., 0] + 1j * zeta[..., 1]
    if not self_pairs:
        wn = np.asarray(w, np.float64)
        xn = np.asarray(x, np.float64)
        q, W, _ = multipoles(piv, nbr, wn, wn * xn * xn, edges, 0, nthreads=nthreads)
        d = ref.self_pair_term(W, q[:, 0, :].real, np.asarray(pv, np.float64))
        z[:, np.arange(nb), np.arange(nb)] -= d[None, :] / np.sum(wp)
    return z, int(pairs[0])


def setup_seconds(nbr, w, x, edges, m_max):
    """Seconds the C oracle spends building its neighbour grid (part of every estimate call)."""
    lib = _load()
    nbr = _c(nbr)
    w = _c(w)
    v = _c(np.asarray(w, np.float64) * np.asarray(x, np.float64))
    edges = _c(edges)
    nx, ny, nz = _c(nbr[0]), _c(nbr[1]), _c(nbr[2])
    t = lib.zo_setup_seconds(nbr.shape[1], _ptr(nx), _ptr(ny), _ptr(nz), _ptr(w), _ptr(v), len(edges) - 1,
                             _ptr(edges), m_max)
    if t < 0:
        raise RuntimeError("zo_setup_seconds failed")
    return t


def estimate_cross(piv, nbr, w, fields, edges, m_max, wp, pivot_fields, cyclic=False, nthreads=0):
    """Multi-field estimator (ref.estimate_cross) with the C oracle's multipoles per field."""
    X = []
    for xf in fields:
        a, W, N = multipoles(piv, nbr, w, xf, edges, m_max, nthreads=nthreads)
        X.append(ref.normalise(a, W))
    terms = [(0, 1, 2), (1, 2, 0), (2, 0, 1)] if cyclic else [(0, 1, 2)]
    wp = np.asarray(wp, np.float64)
    z = 0
    for ia, ib, ic in terms:
        z = z + ref.contract_cross(X[ib], X[ic], wp * np.asarray(pivot_fields[ia], np.float64))
    return z / np.sum(wp), int(N.sum())


def mix64(j):
    """SplitMix64 finaliser of uint64 array j (matches oracle_cpu.c)."""
    v = np.asarray(j, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
    v = (v ^ (v >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    v = (v ^ (v >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return v ^ (v >> np.uint64(31))
