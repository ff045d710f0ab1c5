"""GPU parity of the angular-histogram estimator (z3_index_set_phi_bins,
z3_accumulate_histogram, z3_estimate_histogram) against the oracle's oracle/hist.py:
per-(pivot, radial bin, angular bin) pair counts bit-exact, W and N exact, per-pivot
multipoles within 1e-11 of each bin's scale (FP64; the FP32 storage of the mixed path
within 1.2e-7), zeta within 1e-10 (FP64) and 1e-6 (mixed); the three-point golden values;
full-sky HEALPix pivots at both poles and across the longitude wrap; the bench's largest
configuration (nside512, m_max 64, 130 angular bins) on sampled pivots; m_max up to 127, with
weights and per-cell counts on the widest lane layouts; argument checks."""

import ctypes

import numpy as np
import pytest
import torch

import paper_2408_16847_amd as z3
from paper_2408_16847_amd import _lib
from oracle import hist
from synth import CONFIGS, make_positions, make_values, phi_boundaries, ring_centres
from synth.bins import arcmin, chord2_edges, theta_edges
from tests import gpu_helpers as G
from tests import pins

pytestmark = pytest.mark.gpu


def _gpu_cells(idx, M, p0, p1, prec="fp64", norm="none"):
    out = z3.accumulate_hist(idx, M, p0, p1, prec=prec, norm=norm, want_w=True, want_counts=True,
                             want_counts_phi=True)
    torch.cuda.synchronize()
    A = out["A"].double().cpu().numpy()
    a = np.transpose(A[:, 0] + 1j * A[:, 1], (2, 0, 1))  # [P, m+1, nb]
    return (a, out["W"].cpu().numpy().T, out["counts"].cpu().numpy().T,
            np.transpose(out["counts_phi"].cpu().numpy(), (2, 0, 1)))


def _check_pivots(idx, xyz, x, w, E, M, bnd, p0, p1, perm):
    pm = perm[p0:p1]
    ao, Wo, No, Ho, Co = hist.multipoles_hist(xyz[:, pm], xyz, w, x, E, M, bnd, want_hist=True)
    scale = np.abs(ao).max(axis=1, keepdims=True) + 1e-300
    for prec, tol in (("fp64", 1e-11), ("mixed", 1.2e-7)):
        a, W, N, C = _gpu_cells(idx, M, p0, p1, prec=prec)
        assert np.array_equal(C, Co), prec
        assert np.array_equal(N, No), prec
        assert np.array_equal(W, Wo) or np.abs(W - Wo).max() <= 1e-13 * np.abs(Wo).max(), prec
        err = (np.abs(a - ao) / scale).max()
        G.say("  hist multipoles", prec, "pivots", p0, p1, "cells", int(Co.sum()), "err", err)
        assert err < tol, (prec, err)


@pytest.mark.parametrize("n_phi", [8, 16, 40])
def test_three_point_golden(n_phi):
    G.say("case: histogram three-point", n_phi)
    xyz, E, x = pins.three_point_case()
    gold_pairs, gold = pins.golden_three_point()
    M = min(4, n_phi // 2 - 1)
    idx = G.build(xyz, x, E)
    idx.set_phi_bins(phi_boundaries(n_phi))
    for prec, tol in (("fp64", 1e-14), ("mixed", 1e-6)):
        z, pairs = z3.estimate_hist(idx, M, prec=prec)
        assert pairs == gold_pairs
        assert np.abs(z - gold[:M + 1]).max() < tol
    idx.free()


@pytest.mark.parametrize("n_phi,M", [(8, 3), (24, 10), (64, 31)])
def test_cap_lognormal(n_phi, M):
    G.say("case: histogram cap", n_phi, M)
    cfg = CONFIGS["cap20k"]
    xyz_t = make_positions(cfg)
    x = make_values(cfg, xyz_t).numpy()[:4000]
    xyz = np.ascontiguousarray(xyz_t.numpy()[:, :4000])
    E = cfg.edges_chord2()
    w = np.ones(4000)
    bnd = phi_boundaries(n_phi)
    idx = G.build(xyz, x, E)
    idx.set_phi_bins(bnd)
    perm = G.perm(idx)
    for p0, p1 in ((0, 131), (1900, 2333), (3800, 4000)):
        _check_pivots(idx, xyz, x, w, E, M, bnd, p0, p1, perm)
    zo, po = hist.estimate_hist(xyz, xyz, w, x, E, M, w, x, bnd)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        z, pairs = z3.estimate_hist(idx, M, prec=prec)
        e = G.err_m(z, zo)
        G.say("  hist zeta", prec, "err", e.max())
        assert pairs == po
        assert e.max() < tol
    idx.free()


def test_weighted_ragged_ranges():
    G.say("case: histogram weighted, ragged ranges")
    xyz, w, x = pins.random_cap(3000, 5.0, 43)
    E = pins.small_edges(6, lo=0.05, hi=2.0, log=True)
    bnd = phi_boundaries(30)
    idx = G.build(xyz, x, E, w=w)
    idx.set_phi_bins(bnd)
    perm = G.perm(idx)
    _check_pivots(idx, xyz, x, w, E, 12, bnd, 17, 1290, perm)
    zo, po = hist.estimate_hist(xyz, xyz, w, x, E, 12, w, x, bnd)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        zr = torch.zeros((13, 6, 6, 2), dtype=torch.float64, device="cuda")
        sw = torch.zeros(1, dtype=torch.float64, device="cuda")
        pt = torch.zeros(1, dtype=torch.int64, device="cuda")
        for p0, p1 in ((0, 64), (64, 1999), (1999, 3000)):
            z3.estimate_hist_raw(idx, 12, prec, p0, p1, zeta=zr, pair_total=pt, sum_w=sw)
        torch.cuda.synchronize()
        zc = zr.cpu().numpy() / sw.item()
        assert int(pt.item()) == po
        assert G.err_m(zc[..., 0] + 1j * zc[..., 1], zo).max() < tol
    idx.free()


def test_full_sky_poles_and_wrap():
    """HEALPix Nside 64 (49,152 pixels), 6 log bins 20'-300', 64 angular bins, m <= 31:
    pivot ranges at the north pole, across the longitude wrap near the equator and at the
    south pole, against all pixels."""
    G.say("case: histogram full sky")
    xyz_t = ring_centres(64)
    xyz = xyz_t.numpy()
    x = make_values(CONFIGS["nside512"], xyz_t).numpy()
    E = chord2_edges(theta_edges(arcmin(20.0), arcmin(300.0), 6, True))
    bnd = phi_boundaries(64)
    w = np.ones(xyz.shape[1])
    idx = G.build(xyz, x, E)
    idx.set_phi_bins(bnd)
    perm = G.perm(idx)
    n = len(perm)
    seg = perm[n // 2 - 2000:n // 2 + 2000]
    phi = np.arctan2(xyz[1, seg], xyz[0, seg]) % (2 * np.pi)
    wrap = n // 2 - 2000 + int(np.nonzero(phi[1:] < phi[:-1] - np.pi)[0][0]) + 1
    ranges = [(0, 200), (wrap - 100, wrap + 157), (n - 240, n)]
    for p0, p1 in ranges:
        _check_pivots(idx, xyz, x, w, E, 31, bnd, p0, p1, perm)
    pm = np.concatenate([perm[a:b] for a, b in ranges])
    zo, po = hist.estimate_hist(xyz[:, pm], xyz, w, x, E, 31, np.ones(len(pm)), x[pm], bnd)
    zr = torch.zeros((32, 6, 6, 2), dtype=torch.float64, device="cuda")
    pt = torch.zeros(1, dtype=torch.int64, device="cuda")
    for p0, p1 in ranges:
        z3.estimate_hist_raw(idx, 31, "fp64", p0, p1, zeta=zr, pair_total=pt)
    torch.cuda.synchronize()
    zc = zr.cpu().numpy() / len(pm)
    assert int(pt.item()) == po
    assert G.err_m(zc[..., 0] + 1j * zc[..., 1], zo).max() < 1e-10
    idx.free()


@pytest.mark.parametrize("n_phi,M", [(130, 64), (256, 127)])
def test_large_m(n_phi, M):
    G.say("case: histogram large m", n_phi, M)
    xyz, w, x = pins.random_cap(1500, 4.0, 44)
    E = pins.small_edges(4, lo=0.1, hi=2.0, log=True)
    bnd = phi_boundaries(n_phi)
    idx = G.build(xyz, x, E)
    idx.set_phi_bins(bnd)
    zo, po = hist.estimate_hist(xyz, xyz, np.ones(1500), x, E, M, np.ones(1500), x, bnd)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        z, pairs = z3.estimate_hist(idx, M, prec=prec)
        e = G.err_m(z, zo)
        G.say("  err", prec, e.max())
        assert pairs == po
        assert e.max() < tol
    idx.free()


@pytest.mark.parametrize("n_phi,M", [(130, 64), (256, 127)])
def test_large_m_weighted_cells(n_phi, M):
    """Weighted catalogue on the widest lane layouts (8 and 16 lanes per pivot, whose lanes
    split the bands and sum the pivot's weights): per-pivot multipoles, weights, pair counts
    and per-cell counts on a ragged pivot range."""
    G.say("case: histogram large m, weighted, cells", n_phi, M)
    xyz, w, x = pins.random_cap(1500, 4.0, 45)
    E = pins.small_edges(4, lo=0.1, hi=2.0, log=True)
    bnd = phi_boundaries(n_phi)
    idx = G.build(xyz, x, E, w=w)
    idx.set_phi_bins(bnd)
    perm = G.perm(idx)
    _check_pivots(idx, xyz, x, w, E, M, bnd, 37, 261, perm)
    idx.free()


def test_arguments():
    G.say("case: histogram arguments")
    xyz, E, x = pins.three_point_case()
    idx = G.build(xyz, x, E)
    with pytest.raises(_lib.Zeta3Error):  # no bins yet
        z3.estimate_hist(idx, 2)
    bad = phi_boundaries(16).copy()
    bad[3, 0] += 1e-12
    with pytest.raises(_lib.Zeta3Error):
        idx.set_phi_bins(bad)
    with pytest.raises(_lib.Zeta3Error):
        idx.set_phi_bins(phi_boundaries(512))
    idx.set_phi_bins(phi_boundaries(16))
    with pytest.raises(_lib.Zeta3Error):  # m_max >= n_phi / 2
        z3.estimate_hist(idx, 8)
    zeta = torch.zeros((5, 3, 3, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.Zeta3Error):
        _lib.call("z3_estimate_histogram", idx.handle, 0, 4, 7, 0, 3, ctypes.c_void_p(zeta.data_ptr()),
                  ctypes.c_void_p(0), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert torch.count_nonzero(zeta).item() == 0
    idx.free()
    xy = np.random.default_rng(0).uniform(size=(2, 50))
    pidx = z3.Index(torch.from_numpy(xy).cuda(), np.array([0.01, 0.04]), planar=True)
    with pytest.raises(_lib.Zeta3Error):
        pidx.set_phi_bins(phi_boundaries(16))
    pidx.free()


def _neighbour_subset(xyz, piv, theta_max):
    """Indices of the points within theta_max (plus a margin) of any of the pivots, by a
    chunked dot-product filter: every pair the exact chord test accepts is among them."""
    c = np.cos(theta_max + 1e-6)
    keep = np.zeros(xyz.shape[1], dtype=bool)
    for s in range(0, xyz.shape[1], 1 << 18):
        d = xyz[:, s:s + (1 << 18)].T @ piv
        keep[s:s + (1 << 18)] = (d > c).any(axis=1)
    return np.nonzero(keep)[0]


def test_fullsize_nside512_sampled_pivots():
    """The bench's largest histogram configuration (nside512, m_max 64, 130 angular bins) on
    sampled pivot ranges at the north pole, across the longitude wrap near the equator and
    at the south pole, each against the oracle on the neighbours within reach."""
    cfg = CONFIGS["nside512"]
    M, n_phi = 64, 130
    G.say("case: histogram full size", cfg.name, "m_max", M, "n_phi", n_phi)
    xyz_d = make_positions(cfg, device="cuda")
    x_d = make_values(cfg, xyz_d, seed=0)
    E = cfg.edges_chord2()
    idx = z3.Index(xyz_d, E)
    idx.set_values(x_d)
    bnd = phi_boundaries(n_phi)
    idx.set_phi_bins(bnd)
    xyz, x = xyz_d.cpu().numpy(), x_d.cpu().numpy()
    perm = G.perm(idx)
    n = len(perm)
    lo = n // 2 - 20000
    seg = perm[lo:n // 2 + 20000]
    phi = np.arctan2(xyz[1, seg], xyz[0, seg]) % (2 * np.pi)
    wrap = lo + int(np.nonzero(phi[1:] < phi[:-1] - np.pi)[0][0]) + 1
    theta_max = 2.0 * np.arcsin(np.sqrt(E[-1]) / 2.0)
    for p0, p1 in ((0, 211), (wrap - 100, wrap + 141), (n - 190, n)):
        pm = perm[p0:p1]
        sub = _neighbour_subset(xyz, xyz[:, pm], theta_max)
        ao, Wo, No, Ho, Co = hist.multipoles_hist(xyz[:, pm], xyz[:, sub], np.ones(len(sub)), x[sub], E, M, bnd,
                                                  want_hist=True)
        scale = np.abs(ao).max(axis=1, keepdims=True) + 1e-300
        a, W, N, C = _gpu_cells(idx, M, p0, p1, prec="fp64")
        assert np.array_equal(C, Co) and np.array_equal(N, No) and np.array_equal(W, Wo)
        err = (np.abs(a - ao) / scale).max()
        G.say("  pivots", p0, p1, "neighbours", len(sub), "cells", int(Co.sum()), "err", err)
        assert err < 1e-11, err
    idx.free()
