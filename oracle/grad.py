"""FP64 NumPy gradient of the estimator with respect to the field values -- test
infrastructure only (see oracle/__init__.py).

For a real loss L of the normalised zeta_m(b1, b2), let G_m(b1, b2) = dL/dRe zeta + i dL/dIm zeta.
With v_p = w_p x_p, S = sum_p w_p and X_p(b) = sum_{j in b(p)} c_pj x_j,
c_pj = w_j exp(-i m phi_pj) / W_{p,b} (eqs. Xm.binned, zetamEst), a change of x_k moves
zeta through the pivot factor v_k and through every X_p that contains k:

  dL/dx_k = (1/S) w_k Re sum_m sum_{b1 b2} conj(G(b1,b2)) X_k(b1) conj(X_k(b2))
          + (1/S) sum_{p: k in bin a of p} v_p Re sum_m c_pk D_p(a),
  D_p(a)  = sum_b (conj(G(a, b)) + G(b, a)) conj(X_p(b)).

Written out from the definition; weights are held fixed.  Pivots = the catalogue.
"""

from __future__ import annotations

import numpy as np

from . import ref


def zeta_grad(xyz, w, x, edges, m_max, G):
    xyz = np.asarray(xyz, dtype=np.float64)
    n = xyz.shape[1]
    nb = len(edges) - 1
    a, W, _ = ref.multipoles(xyz, xyz, w, x, edges, m_max)
    X = ref.normalise(a, W)                      # [n, m+1, nb]
    S = np.sum(w)
    G = np.asarray(G, dtype=np.complex128)       # [m+1, nb, nb]
    grad = np.zeros(n)
    # pivot term
    for m in range(m_max + 1):
        q = np.einsum("pa,ab,pb->p", X[:, m, :], np.conj(G[m]), np.conj(X[:, m, :]))
        grad += w * q.real / S
    # neighbour term
    H = np.conj(G) + np.swapaxes(G, 1, 2)       # H_m(a, b) = conj(G(a,b)) + G(b,a)
    D = np.einsum("mab,pmb->pma", H, np.conj(X))  # [n, m+1, nb]
    e_n, e_e = ref.bearing_basis(xyz)
    v = w * x
    for p in range(n):
        b = ref.bin_index(ref.pair_d2(xyz[:, p:p + 1], xyz), edges)[0]
        js = np.nonzero(b >= 0)[0]
        if js.size == 0:
            continue
        bb = b[js]
        delta = xyz[:, js] - xyz[:, p:p + 1]
        phi = ref.bearing(delta, e_n[:, p:p + 1], e_e[:, p:p + 1])
        coef = w[js] / W[p, bb]
        tot = np.zeros(js.size)
        for m in range(m_max + 1):
            c = coef * np.exp(-1j * m * phi)
            tot += (c * D[p, m, bb]).real
        np.add.at(grad, js, v[p] * tot / S)
    return grad
