"""Pins of the angular-histogram oracle (oracle/hist.py), independent of its own code:

* m = 0: the histogram estimator equals the direct estimator exactly (up to rounding),
  since the m = 0 harmonic does not depend on the bearing;
* the bin decision (sign tests against the boundary table on an unnormalised frame)
  equals floor(bearing / dphi) of the direct oracle's normalised bearing for every pair
  not within 1e-9 rad of a boundary;
* histogram + FFT + half-bin phase equals a direct sum of exp(-i m phi_c) over the pairs,
  phi_c the centre of each pair's angular bin, written here with direct trigonometry;
* the three-point worked case (tests/golden/three_point.txt): A sits exactly on the
  boundary of bin 0 and B on a later boundary; the half-open rule and bin centres keep
  the relative angle, so the golden rationals hold;
* per (pivot, bin, m), |X_hist - X_direct| <= (m dphi / 2) sum |g_j| (each pair's bearing
  moves by at most half a bin);
* the error against the direct estimator falls as dphi^2 (bin centres are second order;
  bin starts would be first order).
"""

import math

import numpy as np
import pytest

from oracle import hist, ref
from synth import phi_boundaries
from tests import pins


def _direct_with_centres(piv, nbr, w, x, edges, m_max, bounds):
    """a_{m,b} = sum_j w_j x_j exp(-i m phi_c(j)) with direct trigonometry."""
    n_phi = bounds.shape[0]
    P, nb = piv.shape[1], len(edges) - 1
    b = ref.bin_index(ref.pair_d2(piv, nbr), edges)
    pi, j = np.nonzero(b >= 0)
    N_, E_ = hist.frame_unnormalised(piv)
    u1, u2 = hist.tangent_components(nbr[:, j] - piv[:, pi], N_[:, pi], E_[:, pi])
    k = hist.angular_bin(u1, u2, bounds)
    phic = (k + 0.5) * (2.0 * math.pi / n_phi)
    key = pi * nb + b[pi, j]
    a = np.zeros((P, m_max + 1, nb), dtype=np.complex128)
    wx = w * x
    for m in range(m_max + 1):
        re = np.bincount(key, weights=wx[j] * np.cos(m * phic), minlength=P * nb)
        im = np.bincount(key, weights=-wx[j] * np.sin(m * phic), minlength=P * nb)
        a[:, m] = (re + 1j * im).reshape(P, nb)
    W = np.bincount(key, weights=w[j], minlength=P * nb).reshape(P, nb)
    return a, W


@pytest.mark.parametrize("n_phi", [8, 24, 64])
def test_m0_equals_direct(n_phi):
    xyz, w, x = pins.random_cap(400, 3.0, 11)
    E = pins.small_edges(5, lo=0.1, hi=2.0, log=True)
    z, p = hist.estimate_hist(xyz, xyz, w, x, E, 3, w, x, phi_boundaries(n_phi))
    zd, pd = ref.estimate(xyz, xyz, w, x, E, 3, w, x)
    assert p == pd
    assert pins.rel_err(z[0], zd[0]) < 1e-13


@pytest.mark.parametrize("n_phi", [6, 16, 100])
def test_bins_match_direct_bearing(n_phi):
    xyz, w, x = pins.random_cap(500, 4.0, 12)
    # a pivot at the north pole exercises the x-axis fallback of both frames
    xyz[:, 0] = (0.0, 0.0, 1.0)
    E = pins.small_edges(4, lo=0.1, hi=3.0, log=True)
    b = ref.bin_index(ref.pair_d2(xyz, xyz), E)
    pi, j = np.nonzero(b >= 0)
    N_, E_ = hist.frame_unnormalised(xyz)
    delta = xyz[:, j] - xyz[:, pi]
    k = hist.angular_bin(*hist.tangent_components(delta, N_[:, pi], E_[:, pi]), phi_boundaries(n_phi))
    e_n, e_e = ref.bearing_basis(xyz)
    phi = np.mod(ref.bearing(delta, e_n[:, pi], e_e[:, pi]), 2.0 * math.pi)
    dphi = 2.0 * math.pi / n_phi
    t = phi / dphi
    clear = np.abs(t - np.round(t)) > 1e-9 / dphi
    assert clear.mean() > 0.99 and pi[~clear].size < 10
    assert np.array_equal(k[clear], np.floor(t[clear]).astype(int) % n_phi)


@pytest.mark.parametrize("n_phi,m_max", [(8, 3), (21, 10), (64, 10)])
def test_fft_equals_direct_sum_over_bin_centres(n_phi, m_max):
    xyz, w, x = pins.random_cap(300, 3.0, 13)
    E = pins.small_edges(4, lo=0.1, hi=2.0, log=True)
    bnd = phi_boundaries(n_phi)
    a, W, _ = hist.multipoles_hist(xyz, xyz, w, x, E, m_max, bnd)
    ad, Wd = _direct_with_centres(xyz, xyz, w, x, E, m_max, bnd)
    assert np.array_equal(W, Wd) or pins.rel_err(W, Wd) < 1e-15
    assert pins.rel_err(a, ad) < 1e-12
    z, _ = hist.estimate_hist(xyz, xyz, w, x, E, m_max, w, x, bnd)
    zd = ref.contract(ref.normalise(ad, Wd), w * x) / w.sum()
    assert pins.rel_err(z, zd) < 1e-12


@pytest.mark.parametrize("n_phi", [8, 16, 40])
def test_three_point_golden(n_phi):
    xyz, E, x = pins.three_point_case()
    gold_pairs, gold = pins.golden_three_point()
    m_max = min(4, n_phi // 2 - 1)
    w = np.ones(3)
    z, pairs = hist.estimate_hist(xyz, xyz, w, x, E, m_max, w, x, phi_boundaries(n_phi))
    assert pairs == gold_pairs
    assert np.abs(z - gold[:m_max + 1]).max() < 1e-14


def test_per_pair_phase_bound():
    # sparse catalogue: few pairs per (pivot, bin), so the bound is tight per pair
    xyz, w, x = pins.random_cap(200, 6.0, 14)
    E = pins.small_edges(6, lo=0.2, hi=3.0, log=True)
    n_phi, m_max = 12, 5
    a, W, _ = hist.multipoles_hist(xyz, xyz, w, x, E, m_max, phi_boundaries(n_phi))
    ad, Wd, _ = ref.multipoles(xyz, xyz, w, x, E, m_max)
    g = np.abs(w * x)
    b = ref.bin_index(ref.pair_d2(xyz, xyz), E)
    P, nb = xyz.shape[1], len(E) - 1
    pi, j = np.nonzero(b >= 0)
    sg = np.bincount(pi * nb + b[pi, j], weights=g[j], minlength=P * nb).reshape(P, nb)
    dphi = 2 * math.pi / n_phi
    for m in range(m_max + 1):
        bound = (m * dphi / 2) * sg * (1 + 1e-12) + 1e-14
        assert np.all(np.abs(a[:, m] - ad[:, m]) <= bound), m
    # and the bound is nearly reached somewhere (a pair near a bin edge)
    m = m_max
    assert np.max(np.abs(a[:, m] - ad[:, m]) / np.where(sg > 0, sg, 1)) > 0.5 * (m * dphi / 2)


@pytest.mark.parametrize("n_phi,L,m0", [(8, 5, 3), (16, 3, 5), (30, 4, 7)])
def test_ring_closed_form(n_phi, L, m0):
    """One pivot P = (1, 0, 0) and J = n_phi L neighbours on a circle of radius 0.5 deg at
    bearings phi_j = (k + (l + 1/2) / L) dphi (L per angular bin, symmetric about each
    centre), field x_j = cos(m0 phi_j).  Directly X(m0) = J / 2; with every bearing moved
    to its bin centre X(m0) = (n_phi / 2) sin(m0 dphi / 2) / sin(m0 dphi / (2 L)), so the
    ratio is the Dirichlet factor sin(m0 dphi / 2) / (L sin(m0 dphi / (2 L)))."""
    dphi = 2 * math.pi / n_phi
    k, l = np.meshgrid(np.arange(n_phi), np.arange(L), indexing="ij")
    phi = ((k + (l + 0.5) / L) * dphi).ravel()
    rho = math.radians(0.5)
    P = np.array([1.0, 0.0, 0.0])
    pts = (math.cos(rho) * P[:, None] + math.sin(rho) * (np.cos(phi)[None, :] * np.array([0, 0, 1.0])[:, None]
                                                         + np.sin(phi)[None, :] * np.array([0, 1.0, 0])[:, None]))
    nbr = np.concatenate([P[:, None], pts], axis=1)
    x = np.concatenate([[1.0], np.cos(m0 * phi)])
    w = np.ones(nbr.shape[1])
    E = (2 * np.sin(np.radians([0.4, 0.6]) / 2)) ** 2
    a, W, N = hist.multipoles_hist(P[:, None], nbr, w, x, E, m0, phi_boundaries(n_phi))
    assert N[0, 0] == n_phi * L
    ratio = math.sin(m0 * dphi / 2) / (L * math.sin(m0 * dphi / (2 * L)))
    assert abs(a[0, m0, 0] - (n_phi * L / 2) * ratio) < 1e-11 * n_phi * L
    ad, _, _ = ref.multipoles(P[:, None], nbr, w, x, E, m0)
    assert abs(ad[0, m0, 0] - n_phi * L / 2) < 1e-11 * n_phi * L
