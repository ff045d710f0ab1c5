"""Python binding of libzeta3: argument marshalling only; every step runs in HIP kernels.

Typical use (auto-correlation of one catalogue):

    idx = Index(xyz, edges_chord2, weights=None)   # xyz: [3, n] float64 CUDA tensor
    idx.set_values(x)                               # x: [n] or [nmaps, n] float64 CUDA tensor
    zeta, pairs = estimate(idx, m_max=10, prec="fp64")   # complex128 [m_max+1, nb, nb] (host)
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

PREC = {"fp64": 0, "mixed": 1}
NORM = {"bin": 0, "none": 1}
EST_EXCLUDE_SELF = 1  # Z3_EST_EXCLUDE_SELF


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    return t.to(dtype).contiguous()


class Index:
    """Sky-cell index of a catalogue (z3_build_index); with planar=True, positions [2, n] on
    a plane and squared-distance edges (z3_build_index_planar)."""

    def __init__(self, xyz, edges_chord2, weights=None, cell_size: float = 0.0, planar: bool = False):
        xyz = _dev(xyz)
        if xyz.dim() != 2 or xyz.shape[0] != (2 if planar else 3):
            raise ValueError("positions must be [2, n] on a plane" if planar else "xyz must be [3, n]")
        self.n = int(xyz.shape[1])
        self.planar = planar
        self.edges = np.ascontiguousarray(edges_chord2, dtype=np.float64)
        self.nbins = len(self.edges) - 1
        self._w = None if weights is None else _dev(weights)
        h = ctypes.c_void_p()
        _lib.call("z3_build_index_planar" if planar else "z3_build_index", self.n, _ptr(xyz), _ptr(self._w),
                  self.nbins, self.edges.ctypes.data_as(ctypes.c_void_p), float(cell_size), _stream(),
                  ctypes.byref(h))
        self._h = h
        self.nmaps = 0
        self.n_phi = 0
        self._values = None

    @property
    def handle(self):
        return self._h

    def set_values(self, x):
        x = _dev(x)
        if x.dim() == 1:
            x = x.unsqueeze(0)
        if x.shape[1] != self.n:
            raise ValueError("values must be [nmaps, n]")
        _lib.call("z3_index_set_values", self._h, int(x.shape[0]), _ptr(x), _stream())
        self.nmaps = int(x.shape[0])
        self._values = x  # keep alive until the gather has run
        return self

    def update_values(self, x):
        """Replace the attached maps' values in place (same [nmaps, n] shape): kernels only,
        no host synchronisation or allocation, so it can sit in a captured HIP graph.  The
        caller keeps `x` alive until the stream has run."""
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64 or not x.is_contiguous():
            raise TypeError("update_values needs a contiguous float64 CUDA tensor")
        if x.numel() != self.nmaps * self.n:
            raise ValueError("values must be [nmaps, n] with the attached nmaps")
        _lib.call("z3_index_update_values", self._h, _ptr(x), _stream())
        return self

    def set_phi_bins(self, bounds):
        """Angular bins of the histogram estimator: bounds [n_phi, 2] FP64 boundary
        directions (cos, sin)(2 pi k / n_phi), k = 0..n_phi-1 (z3_index_set_phi_bins)."""
        b = np.ascontiguousarray(bounds, dtype=np.float64)
        if b.ndim != 2 or b.shape[1] != 2:
            raise ValueError("bounds must be [n_phi, 2]")
        _lib.call("z3_index_set_phi_bins", self._h, int(b.shape[0]), b.ctypes.data_as(ctypes.c_void_p))
        self.n_phi = int(b.shape[0])
        return self

    def info(self):
        n = ctypes.c_int64()
        nb = ctypes.c_int()
        nm = ctypes.c_int()
        nbands = ctypes.c_int()
        nc = ctypes.c_int64()
        _lib.call("z3_index_info", self._h, ctypes.byref(n), ctypes.byref(nb), ctypes.byref(nm),
                  ctypes.byref(nbands), ctypes.byref(nc))
        return {"n": n.value, "nbins": nb.value, "nmaps": nm.value, "nbands": nbands.value, "ncells": nc.value}

    def perm(self):
        out = torch.empty(self.n, dtype=torch.int64, device="cuda")
        _lib.call("z3_index_perm", self._h, _ptr(out), _stream())
        return out

    def set_batch_shape(self, waves: int = 0, maps_per_wave: int = 0):
        """MFMA many-map kernel block shape: (waves per block, maps per wave), (0, 0) to autotune."""
        _lib.call("z3_index_set_batch_shape", self._h, int(waves), int(maps_per_wave))

    def batch_shape(self, m_max: int, prec: str = "mixed"):
        """The fixed or tuned (waves, maps per wave) for (m_max, prec); (0, 0) if not tuned yet."""
        w, t = ctypes.c_int(), ctypes.c_int()
        _lib.call("z3_index_batch_shape", self._h, m_max, PREC[prec], ctypes.byref(w), ctypes.byref(t))
        return w.value, t.value

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.current_stream().synchronize()
            _lib.load().z3_index_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def accumulate(idx: Index, m_max: int, p0: int = 0, p1: int | None = None, prec="fp64", norm="bin",
               map_index: int = 0, want_a=True, want_w=False, want_counts=False, want_idhash=False,
               pair_total=None):
    """Per-pivot multipoles for pivots [p0, p1) (index order). Returns a dict of CUDA tensors:
    A [m_max+1, 2, nb, P] (float64 or float32), W [nb, P], counts [nb, P], idhash [nb, P]."""
    p1 = idx.n if p1 is None else p1
    P = p1 - p0
    dev = "cuda"
    out = {}
    adt = torch.float64 if prec == "fp64" else torch.float32
    A = torch.empty((m_max + 1, 2, idx.nbins, P), dtype=adt, device=dev) if want_a else None
    W = torch.empty((idx.nbins, P), dtype=torch.float64, device=dev) if want_w else None
    C = torch.empty((idx.nbins, P), dtype=torch.int64, device=dev) if want_counts else None
    H = torch.empty((idx.nbins, P), dtype=torch.int64, device=dev) if want_idhash else None
    _lib.call("z3_accumulate_multipoles", idx.handle, map_index, m_max, PREC[prec], NORM[norm], p0, p1,
              _ptr(A), _ptr(W), _ptr(C), _ptr(H), _ptr(pair_total), _stream())
    out["A"], out["W"], out["counts"], out["idhash"] = A, W, C, H
    return out


def accumulate_hist(idx: Index, m_max: int, p0: int = 0, p1: int | None = None, prec="fp64", norm="bin",
                    map_index: int = 0, want_a=True, want_w=False, want_counts=False, want_counts_phi=False,
                    pair_total=None):
    """Per-pivot multipoles of the angular-histogram estimator (z3_accumulate_histogram):
    A [m_max+1, 2, nb, P], W [nb, P], counts [nb, P], counts_phi [nb, n_phi, P] (int32)."""
    p1 = idx.n if p1 is None else p1
    P = p1 - p0
    adt = torch.float64 if prec == "fp64" else torch.float32
    A = torch.empty((m_max + 1, 2, idx.nbins, P), dtype=adt, device="cuda") if want_a else None
    W = torch.empty((idx.nbins, P), dtype=torch.float64, device="cuda") if want_w else None
    C = torch.empty((idx.nbins, P), dtype=torch.int64, device="cuda") if want_counts else None
    K = torch.empty((idx.nbins, idx.n_phi, P), dtype=torch.int32, device="cuda") if want_counts_phi else None
    _lib.call("z3_accumulate_histogram", idx.handle, map_index, m_max, PREC[prec], NORM[norm], p0, p1, _ptr(A),
              _ptr(W), _ptr(C), _ptr(K), _ptr(pair_total), _stream())
    return {"A": A, "W": W, "counts": C, "counts_phi": K}


def estimate_hist_raw(idx: Index, m_max: int, prec="fp64", p0: int = 0, p1: int | None = None,
                      map_index: int = 0, zeta=None, pair_total=None, sum_w=None):
    """Enqueue the fused histogram estimator for pivots [p0, p1): zeta += (unnormalised)."""
    p1 = idx.n if p1 is None else p1
    if zeta is None:
        zeta = torch.zeros((m_max + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    _lib.call("z3_estimate_histogram", idx.handle, map_index, m_max, PREC[prec], p0, p1, _ptr(zeta),
              _ptr(pair_total), _stream())
    if sum_w is not None:
        _lib.call("z3_pivot_weight_sum", idx.handle, p0, p1, _ptr(sum_w), _stream())
    return zeta


def estimate_hist(idx: Index, m_max: int, prec="fp64", p0: int = 0, p1: int | None = None, map_index: int = 0):
    """Normalised zeta_m of the histogram estimator (complex128 numpy [m+1, nb, nb]) and the pair count."""
    zeta = torch.zeros((m_max + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    estimate_hist_raw(idx, m_max, prec, p0, p1, map_index, zeta, pairs, sw)
    _lib.call("z3_finalize", 1, m_max, idx.nbins, _ptr(zeta), _ptr(sw), _stream())
    z = zeta.cpu().numpy()
    return z[..., 0] + 1j * z[..., 1], int(pairs.item())


def contract(A, piv_v, m_max: int, nbins: int, prec="fp64", zeta=None):
    """zeta += sum_p v_p X X* over materialised multipoles A [m_max+1, 2, nb, P]."""
    P = int(A.shape[-1])
    if zeta is None:
        zeta = torch.zeros((m_max + 1, nbins, nbins, 2), dtype=torch.float64, device="cuda")
    _lib.call("z3_contract", P, m_max, nbins, PREC[prec], _ptr(A.contiguous()), _ptr(_dev(piv_v)), _ptr(zeta),
              _stream())
    return zeta


def estimate_raw(idx: Index, m_max: int, prec="fp64", p0: int = 0, p1: int | None = None, map_index: int = 0,
                 zeta=None, pair_total=None, sum_w=None, self_pairs: bool = True):
    """Enqueue the fused estimator for pivots [p0, p1): zeta += (unnormalised),
    pair_total += pairs, sum_w += sum of pivot weights. All CUDA tensors; no sync.
    self_pairs=False leaves out the k = j terms of the diagonal (Z3_EST_EXCLUDE_SELF)."""
    p1 = idx.n if p1 is None else p1
    if zeta is None:
        zeta = torch.zeros((m_max + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    flags = 0 if self_pairs else EST_EXCLUDE_SELF
    _lib.call("z3_estimate_ex", idx.handle, map_index, m_max, PREC[prec], flags, p0, p1, _ptr(zeta),
              _ptr(pair_total), _stream())
    if sum_w is not None:
        _lib.call("z3_pivot_weight_sum", idx.handle, p0, p1, _ptr(sum_w), _stream())
    return zeta


def estimate(idx: Index, m_max: int, prec="fp64", p0: int = 0, p1: int | None = None, map_index: int = 0,
             self_pairs: bool = True):
    """zeta_m(b1, b2) normalised by the pivots' total weight, as complex128 numpy [m+1, nb, nb],
    and the number of pairs (self_pairs=False: without the k = j terms)."""
    zeta = torch.zeros((m_max + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    estimate_raw(idx, m_max, prec, p0, p1, map_index, zeta, pairs, sw, self_pairs)
    _lib.call("z3_finalize", 1, m_max, idx.nbins, _ptr(zeta), _ptr(sw), _stream())
    z = zeta.cpu().numpy()
    return z[..., 0] + 1j * z[..., 1], int(pairs.item())


def estimate_cross_raw(idx: Index, maps, m_max: int, prec="fp64", cyclic: bool = False, p0: int = 0,
                       p1: int | None = None, zeta=None, pair_total=None, sum_w=None):
    """Enqueue the multi-field estimator of attached maps (A, B, C) for pivots [p0, p1):
    zeta += sum_p w_p x^A_p X^B(b1) conj X^C(b2) (summed over cyclic permutations if cyclic),
    unnormalised; pair_total and sum_w as in estimate_raw.  No sync."""
    p1 = idx.n if p1 is None else p1
    a, b, c = (int(k) for k in maps)
    if zeta is None:
        zeta = torch.zeros((m_max + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    _lib.call("z3_estimate_cross", idx.handle, a, b, c, 1 if cyclic else 0, m_max, PREC[prec], p0, p1,
              _ptr(zeta), _ptr(pair_total), _stream())
    if sum_w is not None:
        _lib.call("z3_pivot_weight_sum", idx.handle, p0, p1, _ptr(sum_w), _stream())
    return zeta


def estimate_cross(idx: Index, maps, m_max: int, prec="fp64", cyclic: bool = False, p0: int = 0,
                   p1: int | None = None):
    """Normalised multi-field zeta_m as complex128 numpy [m+1, nb, nb], and the pair count."""
    zeta = torch.zeros((m_max + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    estimate_cross_raw(idx, maps, m_max, prec, cyclic, p0, p1, zeta, pairs, sw)
    _lib.call("z3_finalize", 1, m_max, idx.nbins, _ptr(zeta), _ptr(sw), _stream())
    z = zeta.cpu().numpy()
    return z[..., 0] + 1j * z[..., 1], int(pairs.item())


def estimate_maps_raw(idx: Index, m_max: int, prec="fp64", p0: int = 0, p1: int | None = None, zeta=None,
                      pair_total=None, sum_w=None):
    """Enqueue the estimator for every attached map at once: zeta [nmaps, m+1, nb, nb, 2] +=."""
    p1 = idx.n if p1 is None else p1
    if zeta is None:
        zeta = torch.zeros((idx.nmaps, m_max + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    _lib.call("z3_estimate_maps", idx.handle, m_max, PREC[prec], p0, p1, _ptr(zeta), _ptr(pair_total), _stream())
    if sum_w is not None:
        _lib.call("z3_pivot_weight_sum", idx.handle, p0, p1, _ptr(sum_w), _stream())
    return zeta


def estimate_maps(idx: Index, m_max: int, prec="fp64", p0: int = 0, p1: int | None = None):
    """Normalised zeta_m of every attached map: complex128 numpy [nmaps, m+1, nb, nb], and the pair count."""
    zeta = torch.zeros((idx.nmaps, m_max + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    estimate_maps_raw(idx, m_max, prec, p0, p1, zeta, pairs, sw)
    _lib.call("z3_finalize", idx.nmaps, m_max, idx.nbins, _ptr(zeta), _ptr(sw), _stream())
    z = zeta.cpu().numpy()
    return z[..., 0] + 1j * z[..., 1], int(pairs.item())


def estimate_pivots_raw(idx: Index, piv_xyz, piv_x, piv_w=None, m_max: int = 0, prec="fp64", p0: int = 0,
                        p1: int | None = None, map_index: int = 0, zeta=None, pair_total=None, sum_w=None):
    """Enqueue the estimator for an external pivot catalogue (piv_xyz [3, P], piv_x [P],
    piv_w [P] or None) against the index's neighbours: zeta += (unnormalised)."""
    piv_xyz = _dev(piv_xyz)
    piv_x = _dev(piv_x)
    piv_w = None if piv_w is None else _dev(piv_w)
    _check_pivot_rows(idx, piv_xyz)
    P = int(piv_xyz.shape[1])
    p1 = P if p1 is None else p1
    if zeta is None:
        zeta = torch.zeros((m_max + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    _lib.call("z3_estimate_pivots", idx.handle, map_index, P, _ptr(piv_xyz), _ptr(piv_w), _ptr(piv_x), m_max,
              PREC[prec], p0, p1, _ptr(zeta), _ptr(pair_total), _ptr(sum_w), _stream())
    return zeta


def _check_pivot_rows(idx: Index, piv_xyz):
    rows = 2 if getattr(idx, "planar", False) else 3
    if piv_xyz.dim() != 2 or piv_xyz.shape[0] != rows:
        raise ValueError(f"pivot positions must be [{rows}, P] for this index")
    if piv_xyz.shape[1] > 0 and piv_xyz.stride(0) != piv_xyz.shape[1]:
        raise ValueError("pivot positions must be contiguous rows")


def estimate_cross_catalogues(idx_b: Index, idx_c: Index, piv_xyz, piv_x, piv_w=None, m_max: int = 0,
                              prec="fp64", map_b: int = 0, map_c: int = 0, zeta=None, sum_w=None):
    """One term of the multi-field estimator over distinct catalogues: external pivots (field
    A) against neighbour catalogues B (bin b1) and C (bin b2), z3_estimate_cross_catalogues.
    Returns (zeta [m+1, nb, nb, 2] CUDA, unnormalised, +=; pairs with B; pairs with C);
    sum_w (a 1-element CUDA tensor) += the pivots' weights if given."""
    piv_xyz = _dev(piv_xyz)
    piv_x = _dev(piv_x)
    piv_w = None if piv_w is None else _dev(piv_w)
    _check_pivot_rows(idx_b, piv_xyz)
    P = int(piv_xyz.shape[1])
    if zeta is None:
        zeta = torch.zeros((m_max + 1, idx_b.nbins, idx_b.nbins, 2), dtype=torch.float64, device="cuda")
    pb = torch.zeros(1, dtype=torch.int64, device="cuda")
    pc = torch.zeros(1, dtype=torch.int64, device="cuda")
    _lib.call("z3_estimate_cross_catalogues", idx_b.handle, map_b, idx_c.handle, map_c, P, _ptr(piv_xyz),
              _ptr(piv_w), _ptr(piv_x), m_max, PREC[prec], 0, P, _ptr(zeta), _ptr(pb), _ptr(pc), _ptr(sum_w),
              _stream())
    return zeta, int(pb.item()), int(pc.item())


def estimate_pivots(idx: Index, piv_xyz, piv_x, piv_w=None, m_max: int = 0, prec="fp64", p0: int = 0,
                    p1: int | None = None, map_index: int = 0):
    """Normalised zeta_m (complex128 numpy) and the pair count for external pivots."""
    zeta = torch.zeros((m_max + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    estimate_pivots_raw(idx, piv_xyz, piv_x, piv_w, m_max, prec, p0, p1, map_index, zeta, pairs, sw)
    _lib.call("z3_finalize", 1, m_max, idx.nbins, _ptr(zeta), _ptr(sw), _stream())
    z = zeta.cpu().numpy()
    return z[..., 0] + 1j * z[..., 1], int(pairs.item())


def adjoint(idx: Index, G, scale: float, m_max: int, map_index: int = 0, p0: int = 0, p1: int | None = None,
            grad=None):
    """grad_x [n] += dL/dx for G = (dL/dRe zeta, dL/dIm zeta) [m+1, nb, nb, 2] of
    zeta = scale * sum_p v_p X_p X_p^H over pivots [p0, p1)."""
    p1 = idx.n if p1 is None else p1
    if grad is None:
        grad = torch.zeros(idx.n, dtype=torch.float64, device="cuda")
    G = _dev(G)
    _lib.call("z3_adjoint", idx.handle, map_index, m_max, p0, p1, _ptr(G), float(scale), _ptr(grad), _stream())
    return grad


def adjoint_maps(idx: Index, G, scale: float, m_max: int, p0: int = 0, p1: int | None = None, grad=None):
    """grad_x [nmaps, n] += dL/dx for G [nmaps, m+1, nb, nb, 2], every attached map at once
    (multipoles of several maps recomputed together)."""
    p1 = idx.n if p1 is None else p1
    if grad is None:
        grad = torch.zeros((idx.nmaps, idx.n), dtype=torch.float64, device="cuda")
    G = _dev(G)
    _lib.call("z3_adjoint_maps", idx.handle, m_max, p0, p1, _ptr(G), float(scale), _ptr(grad), _stream())
    return grad


class GraphStep:
    """One field-level inference step captured in a HIP graph and replayed: new values of
    every attached map, zeta of all maps (eq. zetamEst, normalised by 1/sum_p w_p), and
    the gradient of L = sum (zeta - target)^2 with respect to the values (the adjoint).

    The index must already hold values of the right shape ([nmaps, n]); the constructor
    runs the step once eagerly (which also tunes the many-map block shape), then captures
    it.  `run(x)` copies x into the static input and replays the graph; the returned zeta
    [nmaps, m+1, nb, nb, 2] and grad [nmaps, n] are the graph's own buffers, overwritten by
    the next run.  Everything inside is kernels (the library's value update, estimator,
    contraction, adjoint, and torch elementwise ops); the library's chunk workspaces are a
    fixed reservation held by the index (z3_index_prepare_capture), so nothing is allocated
    inside the graph.  Replays of graphs captured on one index must not overlap.
    """

    def __init__(self, idx: "Index", m_max: int, target, prec: str = "mixed", stream=None):
        self.idx, self.m_max, self.prec = idx, m_max, prec
        nm, n, nb = idx.nmaps, idx.n, idx.nbins
        self.x = torch.zeros((nm, n), dtype=torch.float64, device="cuda")
        self.target = _dev(target).reshape(nm, m_max + 1, nb, nb, 2).clone()
        self.zeta = torch.zeros((nm, m_max + 1, nb, nb, 2), dtype=torch.float64, device="cuda")
        self.grad = torch.zeros((nm, n), dtype=torch.float64, device="cuda")
        # the pivots' weight sum (positions and weights are fixed): read by z3_finalize on the
        # device inside the graph; the adjoint takes its reciprocal as a host scalar
        self.sum_w = torch.zeros(1, dtype=torch.float64, device="cuda")
        _lib.call("z3_pivot_weight_sum", idx.handle, 0, n, _ptr(self.sum_w), _stream())
        s = float(self.sum_w.item())
        self.scale = 1.0 / s if s != 0.0 else 0.0
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            self._body()  # eager: tunes the block shape, measures the workspace the calls use
        torch.cuda.current_stream().wait_stream(self.stream)
        torch.cuda.synchronize()
        # the captured calls take their workspace from the index, reserved here
        reserved = ctypes.c_size_t()
        _lib.call("z3_index_prepare_capture", idx.handle, 0, ctypes.byref(reserved))
        self.workspace_bytes = reserved.value
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self._body()

    def _body(self):
        self.idx.update_values(self.x)
        self.zeta.zero_()
        _lib.call("z3_estimate_maps", self.idx.handle, self.m_max, PREC[self.prec], 0, self.idx.n,
                  _ptr(self.zeta), _ptr(None), _stream())
        _lib.call("z3_finalize", self.idx.nmaps, self.m_max, self.idx.nbins, _ptr(self.zeta), _ptr(self.sum_w),
                  _stream())
        g = 2.0 * (self.zeta - self.target)  # dL/dzeta
        self.grad.zero_()
        _lib.call("z3_adjoint_maps", self.idx.handle, self.m_max, 0, self.idx.n, _ptr(g), float(self.scale),
                  _ptr(self.grad), _stream())

    def run(self, x):
        self.x.copy_(x.reshape(self.x.shape))
        self.graph.replay()
        return self.zeta, self.grad


class Zeta3Fn(torch.autograd.Function):
    """zeta_m = estimator(x) as a differentiable torch op.

    forward(x, idx, m_max, prec): x [n] or [nmaps, n] field values (catalogue order) are
    attached to `idx`, and the normalised zeta [m+1, nb, nb, 2] (or [nmaps, ...]) is
    returned.  backward runs the library's adjoint kernels (FP64) on the same index, so
    the index must not receive other values between forward and backward.
    """

    @staticmethod
    def forward(ctx, x, idx, m_max, prec="fp64"):
        idx.set_values(x.detach())
        sw = torch.zeros(1, dtype=torch.float64, device="cuda")
        if idx.nmaps > 1:
            zeta = estimate_maps_raw(idx, m_max, prec, sum_w=sw)
        else:
            zeta = estimate_raw(idx, m_max, prec, sum_w=sw)
        # eq. zetamEst's 1/sum_p w_p, on the device
        _lib.call("z3_finalize", idx.nmaps, m_max, idx.nbins, _ptr(zeta), _ptr(sw), _stream())
        ctx.idx, ctx.m_max, ctx.sum_w, ctx.shape = idx, m_max, sw, x.shape
        return zeta

    @staticmethod
    def backward(ctx, g):
        idx = ctx.idx
        g = g.contiguous()
        s = float(ctx.sum_w.item())
        scale = 1.0 / s if s != 0.0 else 0.0
        if len(ctx.shape) == 2:
            grad = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
            adjoint_maps(idx, g, scale, ctx.m_max, grad=grad)
        else:
            grad = adjoint(idx, g, scale, ctx.m_max)
        return grad, None, None, None


def resum(zeta, phi):
    """zeta(b1, b2, phi) from zeta_m (complex [m+1, nb, nb] or a [m+1, nb, nb, 2] tensor)."""
    if not isinstance(zeta, torch.Tensor):
        z = np.asarray(zeta)
        zeta = torch.from_numpy(np.stack([z.real, z.imag], -1).astype(np.float64)).cuda()
    zeta = zeta.contiguous()
    m_max, nb = zeta.shape[0] - 1, zeta.shape[1]
    phi = torch.as_tensor(phi, dtype=torch.float64).cuda().contiguous()
    out = torch.empty((nb, nb, phi.numel()), dtype=torch.float64, device="cuda")
    _lib.call("z3_resum", m_max, nb, _ptr(zeta), int(phi.numel()), _ptr(phi), _ptr(out), _stream())
    return out


FFTLOG_FACTORS = ((0, 0), (1, 1), (1, -1), (2, 0))  # (n, mt) of the four biases, in order


def fftlog_workspace_size(N: int, nchi: int, ntheta: int, models_per_pass: int) -> int:
    """Device bytes z3_fftlog_a_functions needs to process models_per_pass models at once."""
    b = ctypes.c_size_t()
    _lib.call("z3_fftlog_workspace_size", int(N), int(nchi), int(ntheta), int(models_per_pass), ctypes.byref(b))
    return b.value


def fftlog_a_functions(Pk, k_min: float, k_max: float, nu, F, chi_min: float, chi_max: float, theta,
                       workspace=None, out=None):
    """A_0, A_1, A_2 of the modelling appendix for a batch of line-of-sight kernels
    (z3_fftlog_a_functions): Pk [N] on the log-spaced k grid, F [nmodels, nchi] on the
    log-spaced chi grid, theta [T] radians, nu the four biases of FFTLOG_FACTORS.
    Returns a float64 CUDA tensor [nmodels, 3, T, T]."""
    Pk = _dev(Pk)
    F = _dev(F)
    theta = _dev(theta)
    if F.dim() == 1:
        F = F[None]
    nmodels, nchi = int(F.shape[0]), int(F.shape[1])
    T = int(theta.numel())
    nu = np.ascontiguousarray(np.asarray(nu, dtype=np.float64).reshape(4))
    if out is None:
        out = torch.empty((nmodels, 3, T, T), dtype=torch.float64, device="cuda")
    elif tuple(out.shape) != (nmodels, 3, T, T) or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor [nmodels, 3, T, T]")
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _lib.call("z3_fftlog_a_functions", int(Pk.numel()), _ptr(Pk), float(k_min), float(k_max),
              nu.ctypes.data_as(ctypes.c_void_p), nchi, float(chi_min), float(chi_max), nmodels, _ptr(F), T,
              _ptr(theta), _ptr(out), _ptr(workspace), ctypes.c_size_t(ws_bytes), _stream())
    return out


def profile_enable(on=True):
    _lib.call("z3_profile_enable", int(bool(on)))


def profile_read(reset=True):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _lib.call("z3_profile_read", ctypes.byref(n), ctypes.byref(ms), int(bool(reset)))
    return n.value, ms.value


def sync():
    _lib.call("z3_sync", _stream())
