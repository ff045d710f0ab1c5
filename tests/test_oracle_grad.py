"""Pins of the oracle gradient: central finite differences of the oracle's zeta.

For a linear functional L = Re sum conj(G) zeta, zeta is quadratic in each x_k (as a pivot
it enters linearly, as a neighbour through X_p(b1) conj(X_p(b2)), and no point is its own
neighbour), so the central difference is exact up to rounding for any step h.
"""

import numpy as np

from oracle import grad, ref
from tests import pins


def _case(seed, n=180):
    xyz, w, x = pins.random_cap(n, 3.0, seed)
    E = pins.small_edges(5)
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(5, 5, 5)) + 1j * rng.normal(size=(5, 5, 5))
    return xyz, w, x, E, G


def _L(xyz, w, x, E, G):
    z, _ = ref.estimate(xyz, xyz, w, x, E, 4, w, x)
    return float(np.sum(G.real * z.real + G.imag * z.imag))


def test_gradient_matches_central_differences_exactly():
    xyz, w, x, E, G = _case(1)
    g = grad.zeta_grad(xyz, w, x, E, 4, G)
    for k in (0, 7, 55, 123, 179):
        for h in (1.0, 0.25):
            xp = x.copy(); xp[k] += h
            xm = x.copy(); xm[k] -= h
            fd = (_L(xyz, w, xp, E, G) - _L(xyz, w, xm, E, G)) / (2 * h)
            assert abs(fd - g[k]) <= 1e-10 * max(1.0, abs(g[k])), (k, h, fd, g[k])


def test_gradient_of_quadratic_loss():
    xyz, w, x, E, _ = _case(2)
    t = ref.estimate(xyz, xyz, w, x, E, 4, w, x)[0] * 0.7 + 0.01
    z = ref.estimate(xyz, xyz, w, x, E, 4, w, x)[0]
    G = 2.0 * (z - t)                               # L = sum |zeta - t|^2
    g = grad.zeta_grad(xyz, w, x, E, 4, G)

    def L(xx):
        zz = ref.estimate(xyz, xyz, w, xx, E, 4, w, xx)[0]
        return float(np.sum(np.abs(zz - t) ** 2))

    for k in (3, 90):
        h = 1e-4 * np.sqrt(np.mean(x * x))
        xp = x.copy(); xp[k] += h
        xm = x.copy(); xm[k] -= h
        fd = (L(xp) - L(xm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-12), (k, fd, g[k])


def test_gradient_mutation_dropped_pivot_term_is_caught(monkeypatch):
    xyz, w, x, E, G = _case(3, n=120)
    orig = grad.zeta_grad

    def no_pivot_term(xyz_, w_, x_, E_, M_, G_):
        g = orig(xyz_, w_, x_, E_, M_, G_)
        a, W, _ = ref.multipoles(xyz_, xyz_, w_, x_, E_, M_)
        X = ref.normalise(a, W)
        for m in range(M_ + 1):
            q = np.einsum("pa,ab,pb->p", X[:, m], np.conj(G_[m]), np.conj(X[:, m]))
            g = g - w_ * q.real / np.sum(w_)
        return g

    g_bad = no_pivot_term(xyz, w, x, E, 4, G)
    k = 11
    xp = x.copy(); xp[k] += 1.0
    xm = x.copy(); xm[k] -= 1.0
    fd = (_L(xyz, w, xp, E, G) - _L(xyz, w, xm, E, G)) / 2.0
    assert abs(fd - g_bad[k]) > 1e-6 * max(1.0, abs(fd))
