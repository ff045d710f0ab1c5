"""Angular-histogram + Fourier-sum estimator of the binned multipoles -- test
infrastructure only (see oracle/__init__.py).

The complexity discussion of the "3PCF binned estimator" subsection pictures the
multipoles around a pivot as histograms in radial and n_phi angular bins followed by a
Fourier transform over the angular bins (n_phi / 2 multipoles), and proposes FFTs for a
large m_max.  This module writes that estimator out in plain NumPy:

1. pairs and radial bins exactly as ref.multipoles (FP64 chord test, half-open bins);
2. tangent components of the separation delta = r_j - r_p on the UNNORMALISED local
   north N = (-z x, -z y, 1 - z z) (x-axis fallback N = (1 - x x, -x y, -x z) when
   (Nx Nx + Ny Ny) + Nz Nz < 1e-24) and east E = N x r_p, each dot product summed as
   (x + y) + z with every product and sum rounded separately:
       u1 = delta . N,   u2 = delta . E
   (u1, u2) is a positive multiple of the bearing's (cos phi, sin phi), so no square root
   or division enters the bin decision;
3. angular bin: with the boundary table D_k = (c_k, s_k) (synth.phi_boundaries), the pair
   is in bin k iff  c_k u2 - s_k u1 >= 0  and  c_{k+1} u2 - s_{k+1} u1 < 0  (indices mod
   n_phi; each product and the difference rounded once), i.e. its bearing lies in
   [k dphi, (k+1) dphi), dphi = 2 pi / n_phi;
4. histogram H_{p,b,k} = sum over the pairs of radial bin b and angular bin k of w_j x_j;
   W_{p,b}, N_{p,b} as in ref;
5. every pair takes its bin centre's bearing (k + 1/2) dphi:
       a_{m,b}(p) = sum_k H_{p,b,k} exp(-i m (k + 1/2) dphi)
   evaluated with numpy.fft (a discrete Fourier transform over k) and the half-bin phase;
   m_max < n_phi / 2 (the transform is n_phi-periodic in m: a_{m + n_phi} = -a_m);
6. normalisation and contraction exactly as ref (eq. zetamEst).
"""

from __future__ import annotations

import numpy as np

from . import ref


def frame_unnormalised(piv):
    """Unnormalised local north N and east E = N x r_p at each pivot ([3, P] each)."""
    x, y, z = piv
    nx, ny, nz = -z * x, -z * y, 1.0 - z * z
    nn = (nx * nx + ny * ny) + nz * nz
    pole = nn < 1e-24
    ax, ay, az = 1.0 - x * x, -x * y, -x * z
    nx = np.where(pole, ax, nx)
    ny = np.where(pole, ay, ny)
    nz = np.where(pole, az, nz)
    ex = ny * z - nz * y
    ey = nz * x - nx * z
    ez = nx * y - ny * x
    return np.stack([nx, ny, nz]), np.stack([ex, ey, ez])


def tangent_components(delta, N, E):
    """u1 = delta . N and u2 = delta . E, summed as (x + y) + z."""
    u1 = (delta[0] * N[0] + delta[1] * N[1]) + delta[2] * N[2]
    u2 = (delta[0] * E[0] + delta[1] * E[1]) + delta[2] * E[2]
    return u1, u2


def angular_bin(u1, u2, bounds):
    """Angular bin of each (u1, u2) by the sign tests against the boundary table."""
    c = bounds[:, 0][None, :]
    s = bounds[:, 1][None, :]
    left = (c * u2[:, None] - s * u1[:, None]) >= 0.0   # bearing within [theta_k, theta_k + pi)
    hit = left & ~np.roll(left, -1, axis=1)
    if not np.all(hit.sum(axis=1) == 1):
        raise ArithmeticError("angular bin not unique")
    return np.argmax(hit, axis=1)


def fourier_over_bins(H, m_max):
    """sum_k H[..., k] exp(-i m (k + 1/2) dphi) for m = 0..m_max (step 5): an FFT over the
    angular bins, then the half-bin phase exp(-i m dphi / 2)."""
    n_phi = H.shape[-1]
    F = np.fft.fft(H, axis=-1)                      # sum_k H_k exp(-2 pi i m k / n_phi)
    m = np.arange(m_max + 1)
    return F[..., :m_max + 1] * np.exp(-1j * np.pi * m / n_phi)


def multipoles_hist(piv, nbr, w, x, edges, m_max, bounds, block=128, want_hist=False):
    """Per-pivot multipoles from angular histograms: a [P, m_max+1, nb] complex, W [P, nb],
    N [P, nb]; with want_hist also H [P, nb, n_phi] (FP64 sums of w x) and the per-cell
    pair counts C [P, nb, n_phi]."""
    piv = np.asarray(piv, dtype=np.float64)
    nbr = np.asarray(nbr, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.float64)
    bounds = np.asarray(bounds, dtype=np.float64)
    n_phi = bounds.shape[0]
    if not 0 <= m_max < n_phi / 2:
        raise ValueError("need 0 <= m_max < n_phi / 2")
    P, nb = piv.shape[1], len(edges) - 1
    wx = np.asarray(w, np.float64) * np.asarray(x, np.float64)
    N_, E_ = frame_unnormalised(piv)
    H = np.zeros((P, nb, n_phi))
    C = np.zeros((P, nb, n_phi), dtype=np.int64)
    W = np.zeros((P, nb))
    Ncnt = np.zeros((P, nb), dtype=np.int64)
    for s in range(0, P, block):
        e = min(P, s + block)
        b = ref.bin_index(ref.pair_d2(piv[:, s:e], nbr), edges)
        pi, j = np.nonzero(b >= 0)
        if pi.size == 0:
            continue
        bb = b[pi, j]
        delta = nbr[:, j] - piv[:, s + pi]
        u1, u2 = tangent_components(delta, N_[:, s + pi], E_[:, s + pi])
        k = angular_bin(u1, u2, bounds)
        key = (pi * nb + bb) * n_phi + k
        size = (e - s) * nb * n_phi
        H[s:e] = np.bincount(key, weights=wx[j], minlength=size).reshape(e - s, nb, n_phi)
        C[s:e] = np.bincount(key, minlength=size).reshape(e - s, nb, n_phi)
        key2 = pi * nb + bb
        W[s:e] = np.bincount(key2, weights=np.asarray(w, np.float64)[j], minlength=(e - s) * nb).reshape(e - s, nb)
        Ncnt[s:e] = np.bincount(key2, minlength=(e - s) * nb).reshape(e - s, nb)
    a = np.transpose(fourier_over_bins(H, m_max), (0, 2, 1))
    if want_hist:
        return a, W, Ncnt, H, C
    return a, W, Ncnt


def estimate_hist(piv, nbr, w, x, edges, m_max, wp, xp, bounds):
    """zeta_m(b1, b2) of the histogram estimator, normalised by sum_p w_p; plus the pair total."""
    a, W, N = multipoles_hist(piv, nbr, w, x, edges, m_max, bounds)
    X = ref.normalise(a, W)
    z = ref.contract(X, np.asarray(wp, np.float64) * np.asarray(xp, np.float64))
    return z / np.sum(wp), int(N.sum())
