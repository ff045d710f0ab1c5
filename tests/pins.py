"""Shared check functions for the oracle pins (used by the pin and mutation tests).

Each check returns normally when the oracle satisfies the pin and raises
AssertionError otherwise, so a planted mistake can be shown to fail it.
"""

from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np

from oracle import brute, ref


def rel_err(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def three_point_case():
    """P at (1,0,0); A 1 deg due north of P; B 2 deg due east of P (|AB| ~ 2.236 deg)."""
    d1, d2 = math.radians(1.0), math.radians(2.0)
    P = np.array([1.0, 0.0, 0.0])
    A = np.array([math.cos(d1), 0.0, math.sin(d1)])
    B = np.array([math.cos(d2), math.sin(d2), 0.0])
    xyz = np.stack([P, A, B], axis=1)
    th = np.radians([0.9, 1.1, 1.9, 2.1])
    E = (2.0 * np.sin(th / 2.0)) ** 2
    x = np.array([1.3, 0.7, -0.4])
    return xyz, E, x


def three_point_expected(x, m_max):
    """Closed form derived from eqs. Xm.binned and zetamEst for the three-point case.

    Pivot P sees A in bin 0 at bearing 0 and B in bin 2 at bearing pi/2; A and B each
    see only P (in bins 0 and 2).  With unit weights every non-empty bin holds one point,
    so X_m(b) = x_j exp(-i m phi_j), and sum_p w_p = 3.
    """
    xp, xa, xb = x
    z = np.zeros((m_max + 1, 3, 3), dtype=np.complex128)
    for m in range(m_max + 1):
        z[m, 0, 2] = xp * xa * xb * np.exp(1j * m * math.pi / 2) / 3.0
        z[m, 2, 0] = np.conj(z[m, 0, 2])
        z[m, 0, 0] = (xp * xa * xa + xa * xp * xp) / 3.0
        z[m, 2, 2] = (xp * xb * xb + xb * xp * xp) / 3.0
    return z


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_three_point():
    """Hand-derived three-point values of ``golden/three_point.txt`` (exact rationals).

    Returns (ordered pair count, zeta[m][b1][b2] complex128 for m = 0..4).
    """
    z = np.zeros((5, 3, 3), dtype=np.complex128)
    pairs = None
    with open(os.path.join(GOLDEN, "three_point.txt")) as f:
        for line in f:
            tok = line.split()
            if not tok or tok[0].startswith("#"):
                continue
            if tok[0] == "pairs":
                pairs = int(tok[1])
                continue
            m, b1, b2 = (int(t) for t in tok[:3])
            re, im = (float(Fraction(t)) for t in tok[3:5])
            z[m, b1, b2] = complex(re, im)
    return pairs, z


def check_three_point(m_max=4, tol=1e-14):
    xyz, E, x = three_point_case()
    w = np.ones(3)
    z, pairs = ref.estimate(xyz, xyz, w, x, E, m_max, w, x)
    assert pairs == 4, pairs
    exp = three_point_expected(x, m_max)
    err = np.abs(z - exp).max()
    assert err <= tol, err


def random_cap(n, radius_deg, seed):
    rng = np.random.default_rng(seed)
    ca = rng.uniform(math.cos(math.radians(radius_deg)), 1.0, n)
    be = rng.uniform(0.0, 2.0 * math.pi, n)
    sa = np.sqrt((1.0 - ca) * (1.0 + ca))
    xyz = np.stack([ca, sa * np.cos(be), sa * np.sin(be)])
    w = rng.uniform(0.5, 2.0, n)
    x = rng.normal(size=n)
    return xyz, w, x


def small_edges(nb=5, lo=0.2, hi=2.5, log=False):
    from synth.bins import chord2_edges, theta_edges
    return chord2_edges(theta_edges(math.radians(lo), math.radians(hi), nb, log))


def check_brute(n=250, seed=1, m_max=5, tol=1e-12, log=False):
    xyz, w, x = random_cap(n, 3.0, seed)
    E = small_edges(6, log=log)
    z, pairs = ref.estimate(xyz, xyz, w, x, E, m_max, w, x)
    zb, pb = brute.zeta_brute(xyz, xyz, w, x, E, m_max, w, x)
    assert pairs == pb, (pairs, pb)
    err = rel_err(z, zb)
    assert err <= tol, err


def check_brute_no_self(n=250, seed=5, m_max=5, tol=1e-12, log=False):
    """Removal of the k = j terms: ref's subtraction against the triplet sum over k != j."""
    xyz, w, x = random_cap(n, 3.0, seed)
    E = small_edges(6, log=log)
    z, pairs = ref.estimate(xyz, xyz, w, x, E, m_max, w, x, self_pairs=False)
    zb, pb = brute.zeta_brute(xyz, xyz, w, x, E, m_max, w, x, self_pairs=False)
    zs, _ = ref.estimate(xyz, xyz, w, x, E, m_max, w, x)
    assert pairs == pb, (pairs, pb)
    err = rel_err(z, zb)
    assert err <= tol, err
    # the option changes the diagonal only
    nb = len(E) - 1
    off = ~np.eye(nb, dtype=bool)
    assert np.array_equal(z[:, off], zs[:, off])
    assert rel_err(z, zs) > 1e-6


def check_cross_brute(n=220, seed=21, m_max=4, tol=1e-12, cyclic=False):
    """Multi-field estimator: ref's per-field multipoles and cross contraction against the
    triplet sum with the pivot, first and second neighbour carrying fields A, B, C."""
    xyz, w, xa = random_cap(n, 3.0, seed)
    rng = np.random.default_rng(seed + 1)
    fields = (xa, rng.normal(size=n), rng.lognormal(size=n) - 1.0)
    E = small_edges(5)
    z, pairs = ref.estimate_cross(xyz, xyz, w, fields, E, m_max, w, fields, cyclic=cyclic)
    zb, pb = brute.zeta_cross_brute(xyz, xyz, w, fields, E, m_max, w, fields, cyclic=cyclic)
    assert pairs == pb, (pairs, pb)
    err = rel_err(z, zb)
    assert err <= tol, err


def random_square(n, side, seed):
    """n points uniform in a square of the given side, weights in [0.5, 2], normal values."""
    rng = np.random.default_rng(seed)
    xy = rng.uniform(0.0, side, size=(2, n))
    return xy, rng.uniform(0.5, 2.0, n), rng.normal(size=n)


def planar_edges(nb=5, lo=0.2, hi=2.5, log=False):
    """Squared-distance edges of nb bins between lo and hi (plane units)."""
    r = np.geomspace(lo, hi, nb + 1) if log else np.linspace(lo, hi, nb + 1)
    return r * r


def check_brute_planar(n=250, seed=31, m_max=5, tol=1e-12, log=False):
    xy, w, x = random_square(n, 6.0, seed)
    E = planar_edges(6, log=log)
    z, pairs = ref.estimate_planar(xy, xy, w, x, E, m_max, w, x)
    zb, pb = brute.zeta_brute_planar(xy, xy, w, x, E, m_max, w, x)
    assert pairs == pb, (pairs, pb)
    err = rel_err(z, zb)
    assert err <= tol, err


def three_point_planar():
    """P at the origin, A one unit along +y ("north"), B two units along +x ("east"):
    the planar twin of three_point_case (|AB| = sqrt(5) beyond the last edge)."""
    xy = np.array([[0.0, 0.0, 2.0], [0.0, 1.0, 0.0]])
    E = np.array([0.9, 1.1, 1.9, 2.1]) ** 2
    x = np.array([1.3, 0.7, -0.4])
    return xy, E, x


def check_three_point_planar(tol=1e-14):
    xy, E, x = three_point_planar()
    w = np.ones(3)
    z, pairs = ref.estimate_planar(xy, xy, w, x, E, 4, w, x)
    gold_pairs, gold = golden_three_point()
    assert pairs == gold_pairs, pairs
    err = np.abs(z - gold).max()
    assert err <= tol, err


def three_catalogues(seed=91):
    """Three different random catalogues on one 3-degree cap (weights, values)."""
    out = []
    for k, n in enumerate((180, 240, 210)):
        xyz, w, x = random_cap(n, 3.0, seed + k)
        out.append((xyz, w, x))
    return out


def check_cross_catalogues_brute(m_max=4, tol=1e-12):
    (pa, wa, xa), (pb, wb, xb), (pc, wc, xc) = three_catalogues()
    E = small_edges(5)
    z, nb_, nc_ = ref.estimate_cross_catalogues(pa, wa, xa, pb, wb, xb, pc, wc, xc, E, m_max)
    zb, pb_, pc_ = brute.zeta_cross_catalogues_brute(pa, wa, xa, pb, wb, xb, pc, wc, xc, E, m_max)
    assert (nb_, nc_) == (pb_, pc_), ((nb_, nc_), (pb_, pc_))
    err = rel_err(z, zb)
    assert err <= tol, err


def golden_three_point_no_self():
    """The hand-derived three-point values without the k = j terms: every non-empty bin
    of every pivot holds one point, so the diagonal entries vanish and the rest stays."""
    pairs, z = golden_three_point()
    for b in range(z.shape[1]):
        z[:, b, b] = 0.0
    return pairs, z


def check_weight_invariance(seed=2, m_max=4):
    """w -> 2w leaves zeta unchanged exactly (per-bin average and 1/sum w_p)."""
    xyz, w, x = random_cap(200, 3.0, seed)
    E = small_edges(5)
    z1, _ = ref.estimate(xyz, xyz, w, x, E, m_max, w, x)
    z2, _ = ref.estimate(xyz, xyz, 2.0 * w, x, E, m_max, 2.0 * w, x)
    assert np.array_equal(z1, z2), rel_err(z2, z1)


def check_m0_annulus_means(seed=3, tol=1e-13):
    """zeta_0(a, b) = (1/sum w_p) sum_p v_p mean_a(p) mean_b(p), annulus means by bincount."""
    xyz, w, x = random_cap(300, 3.0, seed)
    E = small_edges(6)
    nb = len(E) - 1
    z, _ = ref.estimate(xyz, xyz, w, x, E, 0, w, x)
    exp = np.zeros((nb, nb))
    for p in range(xyz.shape[1]):
        d = xyz - xyz[:, p:p + 1]
        d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        b = np.full(d2.shape, -1)
        for k in range(nb):
            b[(d2 >= E[k]) & (d2 < E[k + 1])] = k
        s = b >= 0
        ws = np.bincount(b[s], weights=w[s], minlength=nb)
        vs = np.bincount(b[s], weights=(w * x)[s], minlength=nb)
        mean = np.where(ws > 0, vs / np.where(ws > 0, ws, 1), 0.0)
        exp += w[p] * x[p] * np.outer(mean, mean)
    exp /= w.sum()
    err = rel_err(z[0].real, exp)
    assert err <= tol, err
    assert np.abs(z[0].imag).max() == 0.0
