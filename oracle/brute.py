"""Brute-force triplet sum -- test infrastructure only (see oracle/__init__.py).

Evaluates the binned estimator as an explicit sum over triangles (pivot p, neighbour j
in bin a, neighbour k in bin b), without any per-pivot reference direction:

    zeta_m(a, b) = (1 / sum_p w_p) sum_p w_p x_p
                   sum_{j in a(p)} sum_{k in b(p)} (w_j x_j / W_{p,a}) (w_k x_k / W_{p,b})
                   exp(-i m (phi_j - phi_k))

which is eq. zetamEst with X_m expanded (the j = k terms included; with
self_pairs=False the triangles with k = j are left out of the sum, the correction of
the diagonal overcount noted in the kappa^3 multipole-signal subsection).  The opening angle
phi_j - phi_k is taken from the tangent vectors t = delta - (delta . r_p) r_p:
cos = t_j . t_k / |t_j||t_k|, sin = r_p . (t_j x t_k) / |t_j||t_k| (angles growing from
north through east).  Because the angle between two neighbours does not depend on n_hat,
this checks the bearing, multipole, normalisation and contraction steps of ref.py
independently.  Cost O(sum_p n_p^2): tiny inputs only.
"""

from __future__ import annotations

import numpy as np


def _bins_by_loop(d2: np.ndarray, edges: np.ndarray) -> np.ndarray:
    b = np.full(d2.shape, -1, dtype=np.int64)
    for k in range(len(edges) - 1):
        b[(d2 >= edges[k]) & (d2 < edges[k + 1])] = k
    return b


def zeta_brute(piv, nbr, w, x, edges, m_max, wp, xp, self_pairs=True):
    piv = np.asarray(piv, dtype=np.float64)
    nbr = np.asarray(nbr, dtype=np.float64)
    nb = len(edges) - 1
    acc = np.zeros((m_max + 1, nb, nb), dtype=np.complex128)
    pairs = 0
    for p in range(piv.shape[1]):
        r = piv[:, p]
        d = nbr - r[:, None]
        d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        b = _bins_by_loop(d2, edges)
        sel = b >= 0
        if not sel.any():
            continue
        pairs += int(sel.sum())
        bj = b[sel]
        t = d[:, sel] - np.outer(r, r @ d[:, sel])
        t = t / np.linalg.norm(t, axis=0)
        Wb = np.zeros(nb)
        np.add.at(Wb, bj, w[sel])
        g = w[sel] * x[sel] / Wb[bj]
        cosd = t.T @ t
        sind = np.cross(t.T[:, None, :], t.T[None, :, :], axis=2) @ r
        dphi = np.arctan2(sind, cosd)
        gg = np.outer(g, g) * (wp[p] * xp[p])
        if not self_pairs:
            np.fill_diagonal(gg, 0.0)  # no triangle with k = j
        key = (bj[:, None] * nb + bj[None, :]).ravel()
        for m in range(m_max + 1):
            ph = np.exp(-1j * m * dphi) * gg
            re = np.bincount(key, weights=ph.real.ravel(), minlength=nb * nb)
            im = np.bincount(key, weights=ph.imag.ravel(), minlength=nb * nb)
            acc[m] += (re + 1j * im).reshape(nb, nb)
    return acc / np.sum(wp), pairs


def zeta_cross_brute(piv, nbr, w, fields, edges, m_max, wp, pivot_fields, cyclic=False):
    """Multi-field triplet sum: pivot p carries field A, neighbour j (bin a) field B and
    neighbour k (bin b) field C,

        zeta_m(a, b) = (1/sum_p w_p) sum_p w_p x^A_p sum_{j in a} sum_{k in b}
                       (w_j x^B_j / W_{p,a}) (w_k x^C_k / W_{p,b}) exp(-i m (phi_j - phi_k)),

    plus, with cyclic=True, the same with (B, C, A) and (C, A, B).  Angles as in zeta_brute.
    """
    piv = np.asarray(piv, dtype=np.float64)
    nbr = np.asarray(nbr, dtype=np.float64)
    nb = len(edges) - 1
    terms = [(0, 1, 2), (1, 2, 0), (2, 0, 1)] if cyclic else [(0, 1, 2)]
    acc = np.zeros((m_max + 1, nb, nb), dtype=np.complex128)
    pairs = 0
    for p in range(piv.shape[1]):
        r = piv[:, p]
        d = nbr - r[:, None]
        d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        b = _bins_by_loop(d2, edges)
        sel = b >= 0
        if not sel.any():
            continue
        pairs += int(sel.sum())
        bj = b[sel]
        t = d[:, sel] - np.outer(r, r @ d[:, sel])
        t = t / np.linalg.norm(t, axis=0)
        Wb = np.zeros(nb)
        np.add.at(Wb, bj, w[sel])
        dphi = np.arctan2(np.cross(t.T[:, None, :], t.T[None, :, :], axis=2) @ r, t.T @ t)
        key = (bj[:, None] * nb + bj[None, :]).ravel()
        for ia, ib, ic in terms:
            gj = w[sel] * fields[ib][sel] / Wb[bj]
            gk = w[sel] * fields[ic][sel] / Wb[bj]
            gg = np.outer(gj, gk) * (wp[p] * pivot_fields[ia][p])
            for m in range(m_max + 1):
                ph = np.exp(-1j * m * dphi) * gg
                re = np.bincount(key, weights=ph.real.ravel(), minlength=nb * nb)
                im = np.bincount(key, weights=ph.imag.ravel(), minlength=nb * nb)
                acc[m] += (re + 1j * im).reshape(nb, nb)
    return acc / np.sum(wp), pairs


def zeta_brute_planar(piv, nbr, w, x, edges, m_max, wp, xp, self_pairs=True):
    """Triplet sum for pivots on a plane: positions [2, n]; the opening angle phi_j - phi_k
    from the separation vectors, cos = d_j . d_k / |d_j||d_k|, sin = (d_j x d_k)_z / |d_j||d_k|
    (angles measured from +y towards +x)."""
    piv = np.asarray(piv, dtype=np.float64)
    nbr = np.asarray(nbr, dtype=np.float64)
    nb = len(edges) - 1
    acc = np.zeros((m_max + 1, nb, nb), dtype=np.complex128)
    pairs = 0
    for p in range(piv.shape[1]):
        dx = nbr[0] - piv[0, p]
        dy = nbr[1] - piv[1, p]
        b = _bins_by_loop(dx * dx + dy * dy, edges)
        sel = b >= 0
        if not sel.any():
            continue
        pairs += int(sel.sum())
        bj = b[sel]
        u, v = dx[sel], dy[sel]
        nrm = np.hypot(u, v)
        u, v = u / nrm, v / nrm
        cosd = np.outer(u, u) + np.outer(v, v)
        sind = np.outer(u, v) - np.outer(v, u)
        dphi = np.arctan2(sind, cosd)
        Wb = np.zeros(nb)
        np.add.at(Wb, bj, w[sel])
        g = w[sel] * x[sel] / Wb[bj]
        gg = np.outer(g, g) * (wp[p] * xp[p])
        if not self_pairs:
            np.fill_diagonal(gg, 0.0)  # no triangle with k = j
        key = (bj[:, None] * nb + bj[None, :]).ravel()
        for m in range(m_max + 1):
            ph = np.exp(-1j * m * dphi) * gg
            re = np.bincount(key, weights=ph.real.ravel(), minlength=nb * nb)
            im = np.bincount(key, weights=ph.imag.ravel(), minlength=nb * nb)
            acc[m] += (re + 1j * im).reshape(nb, nb)
    return acc / np.sum(wp), pairs


def zeta_cross_catalogues_brute(piv, wp, xp, nbr_b, w_b, x_b, nbr_c, w_c, x_c, edges, m_max):
    """Triplet sum over distinct catalogues: pivot p (catalogue A), neighbour j of catalogue
    B in bin a and neighbour k of catalogue C in bin b, each normalised by its own
    catalogue's bin weight, with the opening angle from the tangent vectors at p."""
    piv = np.asarray(piv, dtype=np.float64)
    nb = len(edges) - 1
    acc = np.zeros((m_max + 1, nb, nb), dtype=np.complex128)
    pairs_b = pairs_c = 0

    def side(r, nbr, w, x):
        d = np.asarray(nbr, dtype=np.float64) - r[:, None]
        d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        b = _bins_by_loop(d2, edges)
        sel = b >= 0
        t = d[:, sel] - np.outer(r, r @ d[:, sel])
        t = t / np.linalg.norm(t, axis=0) if sel.any() else t
        Wb = np.zeros(nb)
        np.add.at(Wb, b[sel], w[sel])
        return b[sel], t, w[sel] * x[sel] / np.where(Wb > 0, Wb, 1.0)[b[sel]], int(sel.sum())

    for p in range(piv.shape[1]):
        r = piv[:, p]
        bj, tj, gj, nj = side(r, nbr_b, w_b, x_b)
        bk, tk, gk, nk = side(r, nbr_c, w_c, x_c)
        pairs_b += nj
        pairs_c += nk
        if nj == 0 or nk == 0:
            continue
        cosd = tj.T @ tk
        sind = np.cross(tj.T[:, None, :], tk.T[None, :, :], axis=2) @ r
        dphi = np.arctan2(sind, cosd)
        gg = np.outer(gj, gk) * (wp[p] * xp[p])
        key = (bj[:, None] * nb + bk[None, :]).ravel()
        for m in range(m_max + 1):
            ph = np.exp(-1j * m * dphi) * gg
            re = np.bincount(key, weights=ph.real.ravel(), minlength=nb * nb)
            im = np.bincount(key, weights=ph.imag.ravel(), minlength=nb * nb)
            acc[m] += (re + 1j * im).reshape(nb, nb)
    return acc / np.sum(wp), pairs_b, pairs_c


def dirichlet_resum_brute(piv, nbr, w, x, edges, M, wp, xp, phi):
    """Triplet density smoothed by the Dirichlet kernel D_M(phi - (phi_j - phi_k)).

    sum_{m=-M}^{M} zeta_m exp(i m phi) equals, term by term,
    (1/sum w_p) sum_p v_p sum_jk g_j g_k D_M(phi - phi_jk) with
    D_M(t) = sum_{|m|<=M} exp(i m t) = sin((M + 1/2) t) / sin(t/2).
    Returns [nb, nb, nphi] real.
    """
    piv = np.asarray(piv, dtype=np.float64)
    nbr = np.asarray(nbr, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    nb = len(edges) - 1
    out = np.zeros((nb, nb, phi.size))
    for p in range(piv.shape[1]):
        r = piv[:, p]
        d = nbr - r[:, None]
        d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        b = _bins_by_loop(d2, edges)
        sel = b >= 0
        if not sel.any():
            continue
        bj = b[sel]
        t = d[:, sel] - np.outer(r, r @ d[:, sel])
        t = t / np.linalg.norm(t, axis=0)
        Wb = np.zeros(nb)
        np.add.at(Wb, bj, w[sel])
        g = w[sel] * x[sel] / Wb[bj]
        cosd = t.T @ t
        crs = np.cross(t.T[:, None, :], t.T[None, :, :], axis=2)
        sind = crs @ r
        dphi = np.arctan2(sind, cosd)
        gg = np.outer(g, g) * (wp[p] * xp[p])
        tt = phi[None, None, :] - dphi[:, :, None]
        half = np.sin(tt / 2.0)
        small = np.abs(half) < 1e-12
        kern = np.where(small, 2.0 * M + 1.0, np.sin((M + 0.5) * tt) / np.where(small, 1.0, half))
        contrib = gg[:, :, None] * kern
        for a_ in range(nb):
            ia = bj == a_
            if not ia.any():
                continue
            for b_ in range(nb):
                ib = bj == b_
                if ib.any():
                    out[a_, b_] += contrib[np.ix_(ia, ib)].sum(axis=(0, 1))
    return out / np.sum(wp)
