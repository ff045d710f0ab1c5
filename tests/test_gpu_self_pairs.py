"""GPU parity of the estimator without the k = j terms (Z3_EST_EXCLUDE_SELF).

The paper notes (kappa^3 multipole-signal subsection) that the product X_m(b) conj X_m(b)
counts each neighbour with itself on the diagonal b1 = b2.  z3_estimate_ex removes those
terms; the oracle removes them the same way and is pinned against the brute-force triplet
sum over k != j.  Bars: pair counts exact; per-m max-normalised error against the no-self
estimate's own maximum within 1e-10 (FP64) and 1e-6 (mixed: FP64 multipoles rounded once
to FP32, split-FP32 contraction); entries off the diagonal bit-identical to those of
z3_estimate.
"""

import ctypes

import numpy as np
import pytest
import torch

import paper_2408_16847_amd as z3
from paper_2408_16847_amd import _lib
from oracle import cpu
from synth import CONFIGS, make_positions, make_values
from tests import gpu_helpers as G
from tests import pins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cap():
    cfg = CONFIGS["cap20k"]
    xyz_t = make_positions(cfg)
    x = make_values(cfg, xyz_t).numpy()
    return cfg, xyz_t.numpy(), x


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_three_point_without_self_pairs(prec, tol):
    G.say("case: three-point without self pairs", prec)
    xyz, E, x = pins.three_point_case()
    idx = G.build(xyz, x, E)
    z, pairs = z3.estimate(idx, 4, prec=prec, self_pairs=False)
    gold_pairs, exp = pins.golden_three_point_no_self()
    assert pairs == gold_pairs
    assert np.abs(z - exp).max() < tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_cap20k_without_self_pairs(cap, prec, tol):
    cfg, xyz, x = cap
    G.say("case: cap20k without self pairs", prec)
    E = cfg.edges_chord2()
    w = np.ones(xyz.shape[1])
    idx = G.build(xyz, x, E)
    z, pairs = z3.estimate(idx, cfg.m_max, prec=prec, self_pairs=False)
    # without the k = j terms both paths store and contract FP64 multipoles, so the entries
    # off the diagonal are the FP64 estimate's, bit for bit
    zs, pairs_s = z3.estimate(idx, cfg.m_max, prec="fp64")
    zo, po = cpu.estimate(xyz, xyz, w, x, E, cfg.m_max, w, x, self_pairs=False)
    assert pairs == po == pairs_s
    e = G.err_m(z, zo)
    G.say("err_m", prec, e)
    assert e.max() <= tol, e
    nb = len(E) - 1
    off = ~np.eye(nb, dtype=bool)
    assert np.array_equal(z[:, off], zs[:, off])
    assert np.all(np.diagonal(z, axis1=1, axis2=2).imag == 0)
    # the removed terms are a visible part of the diagonal on this map
    assert np.abs(np.diagonal(z - zs, axis1=1, axis2=2)).max() > 1e-3 * np.abs(zs).max()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_weighted_without_self_pairs_and_pivot_ranges(prec, tol):
    G.say("case: weighted cap without self pairs", prec)
    xyz, w, x = pins.random_cap(3000, 4.0, 37)
    E = pins.small_edges(7, lo=0.05, hi=1.5, log=True)
    idx = G.build(xyz, x, E, w=w)
    z, pairs = z3.estimate(idx, 6, prec=prec, self_pairs=False)
    zo, po = cpu.estimate(xyz, xyz, w, x, E, 6, w, x, self_pairs=False)
    assert pairs == po
    err = G.err_m
    assert err(z, zo).max() <= tol
    # ragged pivot ranges accumulate into one unnormalised zeta
    zr = torch.zeros((7, 7, 7, 2), dtype=torch.float64, device="cuda")
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    pt = torch.zeros(1, dtype=torch.int64, device="cuda")
    for p0, p1 in ((0, 77), (77, 1300), (1300, 3000)):
        z3.estimate_raw(idx, 6, prec, p0, p1, zeta=zr, pair_total=pt, sum_w=sw, self_pairs=False)
    torch.cuda.synchronize()
    zc = zr.cpu().numpy() / sw.item()
    assert int(pt.item()) == po
    assert err(zc[..., 0] + 1j * zc[..., 1], zo).max() <= tol


def test_unknown_flags_rejected():
    G.say("case: z3_estimate_ex flags")
    xyz, E, x = pins.three_point_case()
    idx = G.build(xyz, x, E)
    zeta = torch.zeros((5, 3, 3, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.Zeta3Error) as ei:
        _lib.call("z3_estimate_ex", idx.handle, 0, 4, 0, 2, 0, 3, ctypes.c_void_p(zeta.data_ptr()),
                  ctypes.c_void_p(0), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert ei.value.status == 1
    torch.cuda.synchronize()
    assert torch.count_nonzero(zeta).item() == 0
