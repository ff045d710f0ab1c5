"""Plain NumPy FP64 estimator -- test infrastructure only (see oracle/__init__.py).

Follows the binned estimator of the paper's "3PCF binned estimator" subsection step by
step, with direct trigonometry (no recurrences), O(N_pivots x N) pair tests.
Arrays: positions are [3, n] FP64 unit vectors; per-pivot outputs are [P, m_max+1, nb].
"""

from __future__ import annotations

import numpy as np


def pair_d2(piv: np.ndarray, nbr: np.ndarray) -> np.ndarray:
    """Squared chord between each pivot and each neighbour, [P, N].

    d2 = (dx*dx + dy*dy) + dz*dz with dx = x_j - x_p: elementwise NumPy operations,
    each rounded to nearest separately (the binning-function Theta of eq. Xm.binned
    applied to the chord, which is monotone in the angular distance).
    """
    dx = nbr[0][None, :] - piv[0][:, None]
    dy = nbr[1][None, :] - piv[1][:, None]
    dz = nbr[2][None, :] - piv[2][:, None]
    return (dx * dx + dy * dy) + dz * dz


def bin_index(d2: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """Bin of each squared chord: b with E_b <= d2 < E_{b+1}, else -1 (outside)."""
    nb = len(edges) - 1
    b = np.searchsorted(edges, d2, side="right") - 1
    b[(b < 0) | (b >= nb)] = -1
    return b


def bearing_basis(piv: np.ndarray):
    """Local north and east unit vectors at each pivot, [3, P] each.

    The polar angle of the plane-wave expansion (eq. Xmdef) is measured from an
    arbitrary direction n_hat; here n_hat is local north, and angles grow towards east.
    """
    x, y, z = piv
    nvec = np.stack([-z * x, -z * y, 1.0 - z * z])
    norm = np.sqrt((nvec * nvec).sum(0))
    alt = np.stack([1.0 - x * x, -x * y, -x * z])  # x-axis fallback at the poles
    alt_norm = np.sqrt((alt * alt).sum(0))
    use_alt = norm < 1e-12
    nvec = np.where(use_alt, alt, nvec)
    norm = np.where(use_alt, alt_norm, norm)
    e_n = nvec / norm
    e_e = np.cross(e_n.T, piv.T).T
    return e_n, e_e


def bearing(delta: np.ndarray, e_n: np.ndarray, e_e: np.ndarray) -> np.ndarray:
    """Position angle atan2(delta . e_E, delta . e_N) of each separation vector."""
    u1 = (delta * e_n).sum(0)
    u2 = (delta * e_e).sum(0)
    return np.arctan2(u2, u1)


def multipoles(piv, nbr, w, x, edges, m_max, block=128):
    """Raw binned multipoles of every pivot.

    Returns a [P, m_max+1, nb] complex (a = sum w x exp(-i m phi)), W [P, nb],
    N [P, nb] int64.  (eqs. Xm.binned and Ym/Zm.binned without the normaliser.)
    """
    piv = np.asarray(piv, dtype=np.float64)
    nbr = np.asarray(nbr, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.float64)
    P, nb = piv.shape[1], len(edges) - 1
    a = np.zeros((P, m_max + 1, nb), dtype=np.complex128)
    W = np.zeros((P, nb))
    N = np.zeros((P, nb), dtype=np.int64)
    wx = w * x
    e_n, e_e = bearing_basis(piv)
    for s in range(0, P, block):
        e = min(P, s + block)
        b = bin_index(pair_d2(piv[:, s:e], nbr), edges)
        pi, j = np.nonzero(b >= 0)
        if pi.size == 0:
            continue
        bb = b[pi, j]
        delta = nbr[:, j] - piv[:, s + pi]
        phi = bearing(delta, e_n[:, s + pi], e_e[:, s + pi])
        key = pi * nb + bb
        size = (e - s) * nb
        W[s:e] = np.bincount(key, weights=w[j], minlength=size).reshape(e - s, nb)
        N[s:e] = np.bincount(key, minlength=size).reshape(e - s, nb)
        for m in range(m_max + 1):
            re = np.bincount(key, weights=wx[j] * np.cos(m * phi), minlength=size)
            im = np.bincount(key, weights=-wx[j] * np.sin(m * phi), minlength=size)
            a[s:e, m] = (re + 1j * im).reshape(e - s, nb)
    return a, W, N


def normalise(a, W):
    """X_m(b; p) = a_{m,b}(p) / W_{p,b}; 0 where the bin holds no weight."""
    Wb = W[:, None, :]
    safe = np.where(Wb > 0, Wb, 1.0)
    return np.where(Wb > 0, a / safe, 0.0)


def contract(X, vp):
    """Unnormalised sum_p v_p X_m(b1; p) conj(X_m(b2; p)) -> [m_max+1, nb, nb] (eq. zetamEst).

    Written with real arithmetic, (r1 + i i1)(r2 - i i2) = (r1 r2 + i1 i2) + i (i1 r2 - r1 i2),
    each product rounded separately, so that entry (b2, b1) is exactly the conjugate of
    entry (b1, b2) and the diagonal is exactly real.
    """
    P, M1, nb = X.shape
    re = np.zeros((M1, nb, nb))
    im = np.zeros((M1, nb, nb))
    for p in range(P):
        r = X[p].real
        i = X[p].imag
        re += vp[p] * (r[:, :, None] * r[:, None, :] + i[:, :, None] * i[:, None, :])
        im += vp[p] * (i[:, :, None] * r[:, None, :] - r[:, :, None] * i[:, None, :])
    return re + 1j * im


def self_pair_term(W, Q, vp):
    """The k = j terms of sum_p v_p X_m(b; p) conj(X_m(b; p)), per bin b ([nb], real).

    With X_m(b; p) = sum_{j in b} g_j exp(-i m phi_j), g_j = w_j x_j / W_{p,b}, the product
    X conj X holds sum_j g_j^2 (the same for every m): summed over pivots with the weight
    v_p this is sum_p v_p Q_{p,b} / W_{p,b}^2, Q_{p,b} = sum_{j in b} (w_j x_j)^2 (0 where
    W_{p,b} = 0).  This is the overcount on the diagonal that the paper notes in the kappa^3
    multipole-signal subsection.
    """
    safe = np.where(W > 0, W, 1.0)
    return np.where(W > 0, Q / (safe * safe), 0.0).T @ vp


def estimate(piv, nbr, w, x, edges, m_max, wp, xp, self_pairs=True, planar=False):
    """zeta_m(b1, b2) for the given pivot set, normalised by sum_p w_p; plus the pair total.

    self_pairs=False removes the k = j terms from the diagonal b1 = b2 (self_pair_term);
    planar=True takes positions [2, n] on a plane (multipoles_planar).
    """
    multipoles_ = multipoles_planar if planar else multipoles
    a, W, N = multipoles_(piv, nbr, w, x, edges, m_max)
    X = normalise(a, W)
    z = contract(X, wp * xp)
    if not self_pairs:
        w = np.asarray(w, dtype=np.float64)
        x = np.asarray(x, dtype=np.float64)
        # Q_{p,b} = sum_{j in b} w_j (w_j x_j^2): the m = 0 sum of the field w x^2
        q, _, _ = multipoles_(piv, nbr, w, w * x * x, edges, 0)
        d = self_pair_term(W, q[:, 0, :].real, wp * xp)
        nb = W.shape[1]
        z[:, np.arange(nb), np.arange(nb)] -= d[None, :]
    return z / np.sum(wp), int(N.sum())


def contract_cross(Xa, Xb, vp):
    """Unnormalised sum_p v_p Xa_m(b1; p) conj(Xb_m(b2; p)) -> [m_max+1, nb, nb]: the
    contraction of eq. zetamEst with the two neighbour fields of a cross-correlation."""
    M1, nb = Xa.shape[1], Xa.shape[2]
    out = np.zeros((M1, nb, nb), dtype=np.complex128)
    for p in range(Xa.shape[0]):
        out += vp[p] * (Xa[p][:, :, None] * np.conj(Xb[p][:, None, :]))
    return out


def estimate_cross(piv, nbr, w, fields, edges, m_max, wp, pivot_fields, cyclic=False, planar=False):
    """Multi-field estimator (remark after eq. ubEstimator): the pivot carries field A, the
    bin b1 field B and the bin b2 field C,

        zeta^{A;BC}_m(b1, b2) = (1/sum_p w_p) sum_p w_p x^A_p X^B_m(b1; p) conj(X^C_m(b2; p));

    with cyclic=True the sum over the cyclic permutations (A;BC) + (B;CA) + (C;AB).
    fields = (xA, xB, xC) on the neighbour catalogue, pivot_fields the same on the pivots.
    Returns (zeta [m_max+1, nb, nb], pair total).
    """
    X = []
    for xf in fields:
        a, W, N = (multipoles_planar if planar else multipoles)(piv, nbr, w, xf, edges, m_max)
        X.append(normalise(a, W))
    terms = [(0, 1, 2), (1, 2, 0), (2, 0, 1)] if cyclic else [(0, 1, 2)]
    z = 0
    for ia, ib, ic in terms:
        z = z + contract_cross(X[ib], X[ic], wp * pivot_fields[ia])
    return z / np.sum(wp), int(N.sum())


def planar_bearing(dx, dy):
    """Angle of a separation on the plane, from the +y axis towards +x."""
    return np.arctan2(dx, dy)


def multipoles_planar(piv, nbr, w, x, edges, m_max, block=128):
    """Raw binned multipoles for pivots on a plane (the estimator is the same on any smooth
    manifold, as the paper notes in its description of the code): positions [2, n] (x, y),
    d2 = dx*dx + dy*dy rounded as written, the angle phi = atan2(dx, dy) measured from the +y
    axis towards +x (the plane's "north" and "east").  Returns a, W, N as multipoles()."""
    piv = np.asarray(piv, dtype=np.float64)
    nbr = np.asarray(nbr, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.float64)
    P, nb = piv.shape[1], len(edges) - 1
    a = np.zeros((P, m_max + 1, nb), dtype=np.complex128)
    W = np.zeros((P, nb))
    N = np.zeros((P, nb), dtype=np.int64)
    wx = w * x
    for s in range(0, P, block):
        e = min(P, s + block)
        dx = nbr[0][None, :] - piv[0][s:e, None]
        dy = nbr[1][None, :] - piv[1][s:e, None]
        b = bin_index(dx * dx + dy * dy, edges)
        pi, j = np.nonzero(b >= 0)
        if pi.size == 0:
            continue
        bb = b[pi, j]
        phi = planar_bearing(dx[pi, j], dy[pi, j])
        key = pi * nb + bb
        size = (e - s) * nb
        W[s:e] = np.bincount(key, weights=w[j], minlength=size).reshape(e - s, nb)
        N[s:e] = np.bincount(key, minlength=size).reshape(e - s, nb)
        for m in range(m_max + 1):
            re = np.bincount(key, weights=wx[j] * np.cos(m * phi), minlength=size)
            im = np.bincount(key, weights=-wx[j] * np.sin(m * phi), minlength=size)
            a[s:e, m] = (re + 1j * im).reshape(e - s, nb)
    return a, W, N


def estimate_planar(piv, nbr, w, x, edges, m_max, wp, xp):
    """zeta_m(b1, b2) for pivots on a plane (multipoles_planar), normalised by sum_p w_p."""
    a, W, N = multipoles_planar(piv, nbr, w, x, edges, m_max)
    z = contract(normalise(a, W), wp * xp) / np.sum(wp)
    return z, int(N.sum())


def estimate_cross_catalogues(piv, wp, xp, nbr_b, w_b, x_b, nbr_c, w_c, x_c, edges, m_max):
    """One term of the multi-field estimator over distinct catalogues: pivots (piv, wp, xp)
    carry field A; X^B(b1) is the bin average of catalogue B around each pivot, X^C(b2) that
    of catalogue C:  (1/sum_p w_p) sum_p w_p x_p X^B_m(b1; p) conj(X^C_m(b2; p)).
    Returns (zeta, pairs with B, pairs with C).  The cyclic sum rotates the roles."""
    a_b, W_b, N_b = multipoles(piv, nbr_b, w_b, x_b, edges, m_max)
    a_c, W_c, N_c = multipoles(piv, nbr_c, w_c, x_c, edges, m_max)
    z = contract_cross(normalise(a_b, W_b), normalise(a_c, W_c), np.asarray(wp) * np.asarray(xp))
    return z / np.sum(wp), int(N_b.sum()), int(N_c.sum())


def resum(zeta, phi):
    """zeta(b1, b2, phi) = sum_{m=-M}^{M} zeta_m exp(i m phi), zeta_{-m} = conj(zeta_m).

    (eq. eq_zeta_harmonic truncated at |m| <= M.)  Returns [nb, nb, nphi] real.
    """
    M1 = zeta.shape[0]
    phi = np.asarray(phi, dtype=np.float64)
    out = np.zeros(zeta.shape[1:] + phi.shape, dtype=np.complex128)
    for m in range(-(M1 - 1), M1):
        zm = zeta[m] if m >= 0 else np.conj(zeta[-m])
        out += zm[:, :, None] * np.exp(1j * m * phi)[None, None, :]
    return out.real
