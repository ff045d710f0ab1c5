"""z3_estimate_static (the fused estimator on a static device workspace: no allocation)
against z3_estimate_ex through the C ABI, on two calls in a row, the second with a smaller
input: pair totals equal, zeta within the precision's bar (1e-10 FP64, 1e-6 mixed; the two
entry points sum their pivot chunks in different places)."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2408_16847_amd import _lib
from paper_2408_16847_amd.zeta3 import PREC, EST_EXCLUDE_SELF
from synth import CONFIGS, make_values, ring_centres
from synth.bins import arcmin, chord2_edges, theta_edges
from tests import gpu_helpers as G
from tests import pins

pytestmark = pytest.mark.gpu


def _call(name, idx, M, prec, flags, p0, p1):
    zeta = torch.zeros((M + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    _lib.call(name, idx.handle, 0, M, PREC[prec], flags, p0, p1, ctypes.c_void_p(zeta.data_ptr()),
              ctypes.c_void_p(pairs.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    z = zeta.cpu().numpy()
    return z[..., 0] + 1j * z[..., 1], int(pairs.item())


def _compare(idx, M, prec, tol, flags, p0, p1):
    zs, ps = _call("z3_estimate_static", idx, M, prec, flags, p0, p1)
    ze, pe = _call("z3_estimate_ex", idx, M, prec, flags, p0, p1)
    e = G.err_m(zs, ze).max()
    G.say("  static vs estimate_ex", prec, "flags", flags, "pivots", p0, p1, "pairs", ps, pe, "err", e)
    assert ps == pe and ps > 0
    assert e <= tol
    assert np.abs(zs).max() > 0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_static_workspace_matches_estimate_ex(prec, tol):
    # first call: HEALPix Nside 256 (786,432 pixels), 20 log bins 5'-200', m <= 10: several
    # chunks of the static workspace (~151,000 pivots per chunk in FP64, ~299,000 mixed)
    G.say("case: static workspace, Nside 256", prec)
    xyz_t = ring_centres(256)
    x = make_values(CONFIGS["nside512"], xyz_t).numpy()
    E = chord2_edges(theta_edges(arcmin(5.0), arcmin(200.0), 20, True))
    idx = G.build(xyz_t.numpy(), x, E)
    _compare(idx, 10, prec, tol, 0, 0, idx.n)
    idx.free()
    # second call, smaller: a weighted 3,000-point cap, 7 bins, a ragged pivot range,
    # without the k = j terms (the static workspace still holds the first call's data)
    G.say("case: static workspace, weighted cap", prec)
    xyz, w, xc = pins.random_cap(3000, 4.0, 37)
    idx2 = G.build(xyz, xc, pins.small_edges(7, lo=0.05, hi=1.5, log=True), w=w)
    _compare(idx2, 6, prec, tol, EST_EXCLUDE_SELF, 77, 2901)
    idx2.free()
