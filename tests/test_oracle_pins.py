"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

P1 brute-force triplets, P2 closed-form three-point case, P3 Hermitian structure,
P4 field / weight scaling, P5 reference-direction invariance, P6 rotation and mirror,
P8 m = 0 annulus means, P9 Dirichlet-kernel resummation, P10 brute-force pair counts,
P11 vanishing 3PCF of a Gaussian field, plus C oracle == NumPy reference.
"""

import math

import numpy as np
import pytest

from oracle import brute, cpu, ref
from tests import pins


def test_p2_three_point_closed_form():
    pins.check_three_point()


def test_p2_three_point_values_printed_in_the_derivation():
    # Im zeta_1(0, 2) = x_P x_A x_B / 3 and zeta_m(0, 0) = (x_P x_A^2 + x_A x_P^2) / 3
    xyz, E, x = pins.three_point_case()
    w = np.ones(3)
    z, _ = ref.estimate(xyz, xyz, w, x, E, 2, w, x)
    assert abs(z[1, 0, 2].imag - (-0.364 / 3.0)) < 1e-14
    assert abs(z[1, 0, 0].real - 1.82 / 3.0) < 1e-14
    assert abs(z[0, 2, 2].real - (-0.468 / 3.0)) < 1e-14


def test_p2_three_point_golden_fixture():
    # the closed form used by the other checks against the hand-derived rationals
    pairs, gold = pins.golden_three_point()
    xyz, E, x = pins.three_point_case()
    w = np.ones(3)
    assert pairs == 4
    assert np.abs(pins.three_point_expected(x, 4) - gold).max() < 1e-15
    z, p = ref.estimate(xyz, xyz, w, x, E, 4, w, x)
    assert p == pairs
    assert np.abs(z - gold).max() < 1e-14


def test_p2_three_point_c_oracle_and_brute():
    xyz, E, x = pins.three_point_case()
    w = np.ones(3)
    exp = pins.three_point_expected(x, 4)
    zc, pc = cpu.estimate(xyz, xyz, w, x, E, 4, w, x)
    zb, pb = brute.zeta_brute(xyz, xyz, w, x, E, 4, w, x)
    assert pc == pb == 4
    assert np.abs(zc - exp).max() < 1e-14
    assert np.abs(zb - exp).max() < 1e-14


def test_bearing_convention_north_east():
    # neighbours displaced due north / east / south / west of (1,0,0)
    piv = np.array([[1.0], [0.0], [0.0]])
    e_n, e_e = ref.bearing_basis(piv)
    d = math.radians(0.5)
    nbrs = {0.0: [math.cos(d), 0, math.sin(d)], math.pi / 2: [math.cos(d), math.sin(d), 0],
            math.pi: [math.cos(d), 0, -math.sin(d)], -math.pi / 2: [math.cos(d), -math.sin(d), 0]}
    for phi, r in nbrs.items():
        delta = (np.array(r) - piv[:, 0])[:, None]
        got = ref.bearing(delta, e_n, e_e)[0]
        assert abs(math.remainder(got - phi, 2 * math.pi)) < 1e-12, (phi, got)


@pytest.mark.parametrize("seed,log", [(1, False), (7, True), (11, False)])
def test_p1_brute_random_catalogues(seed, log):
    pins.check_brute(seed=seed, log=log)


@pytest.mark.parametrize("seed,log", [(5, False), (13, True)])
def test_no_self_pairs_brute(seed, log):
    pins.check_brute_no_self(seed=seed, log=log)


@pytest.mark.parametrize("cyclic", [False, True])
def test_cross_fields_brute(cyclic):
    pins.check_cross_brute(cyclic=cyclic)


def test_cross_catalogues_brute():
    pins.check_cross_catalogues_brute()


def test_cross_catalogues_reduce_to_one_catalogue():
    # all three roles on one catalogue: the single-catalogue estimator
    xyz, w, x = pins.random_cap(250, 3.0, 97)
    E = pins.small_edges(5)
    z, p = ref.estimate(xyz, xyz, w, x, E, 4, w, x)
    zc, pb, pc = ref.estimate_cross_catalogues(xyz, w, x, xyz, w, x, xyz, w, x, E, 4)
    assert p == pb == pc
    assert pins.rel_err(zc, z) < 1e-13


def test_cross_fields_special_cases():
    # one field in all three roles: the single term is zeta, the cyclic sum 3 zeta; exchanging
    # the two neighbour fields conjugates and transposes
    xyz, w, x = pins.random_cap(300, 3.0, 23)
    y = np.random.default_rng(24).normal(size=300)
    E = pins.small_edges(5)
    z, p = ref.estimate(xyz, xyz, w, x, E, 4, w, x)
    z1, p1 = ref.estimate_cross(xyz, xyz, w, (x, x, x), E, 4, w, (x, x, x))
    z3_, p3 = ref.estimate_cross(xyz, xyz, w, (x, x, x), E, 4, w, (x, x, x), cyclic=True)
    assert p == p1 == p3
    assert pins.rel_err(z1, z) < 1e-13 and pins.rel_err(z3_, 3.0 * z) < 1e-13
    zbc, _ = ref.estimate_cross(xyz, xyz, w, (x, y, x), E, 4, w, (x, y, x))
    zcb, _ = ref.estimate_cross(xyz, xyz, w, (x, x, y), E, 4, w, (x, x, y))
    assert pins.rel_err(zcb, np.conj(np.swapaxes(zbc, 1, 2))) < 1e-13


@pytest.mark.parametrize("seed,log", [(31, False), (33, True)])
def test_planar_brute(seed, log):
    pins.check_brute_planar(seed=seed, log=log)


def test_planar_three_point_golden():
    pins.check_three_point_planar()


def test_planar_self_pairs_and_fields_brute():
    # the planar options follow the same pins as on the sphere: k != j and three fields
    xy, w, x = pins.random_square(200, 6.0, 37)
    y = np.random.default_rng(38).normal(size=200)
    E = pins.planar_edges(5)
    z, p = ref.estimate(xy, xy, w, x, E, 4, w, x, self_pairs=False, planar=True)
    zs, _ = ref.estimate_planar(xy, xy, w, x, E, 4, w, x)
    zb, pb = brute.zeta_brute_planar(xy, xy, w, x, E, 4, w, x)
    assert p == pb and pins.rel_err(zs, zb) < 1e-12
    zbn, _ = brute.zeta_brute_planar(xy, xy, w, x, E, 4, w, x, self_pairs=False)
    assert pins.rel_err(z, zbn) < 1e-12
    zc, _ = ref.estimate_cross(xy, xy, w, (x, x, x), E, 4, w, (x, x, x), planar=True)
    assert pins.rel_err(zc, zs) < 1e-13
    zc2, _ = ref.estimate_cross(xy, xy, w, (x, y, x), E, 4, w, (x, y, x), planar=True)
    zc3, _ = ref.estimate_cross(xy, xy, w, (x, x, y), E, 4, w, (x, x, y), planar=True)
    assert pins.rel_err(zc3, np.conj(np.swapaxes(zc2, 1, 2))) < 1e-13


def test_planar_rotation_and_mirror():
    # a rotation of the plane keeps zeta; a mirror keeps Re and flips Im (where the pair
    # counts agree, i.e. no pair moved across a bin edge by rounding)
    xy, w, x = pins.random_square(400, 6.0, 35)
    E = pins.planar_edges(5)
    z, p = ref.estimate_planar(xy, xy, w, x, E, 4, w, x)
    a = 0.7
    R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    zr, pr = ref.estimate_planar(R @ xy, R @ xy, w, x, E, 4, w, x)
    mir = np.array([[-1.0], [1.0]]) * xy
    zm, pm = ref.estimate_planar(mir, mir, w, x, E, 4, w, x)
    assert p == pr == pm
    assert pins.rel_err(zr, z) < 1e-10
    assert pins.rel_err(zm, np.conj(z)) < 1e-12


def test_no_self_pairs_three_point_and_c_oracle():
    pairs, gold = pins.golden_three_point_no_self()
    xyz, E, x = pins.three_point_case()
    w = np.ones(3)
    for z, p in (ref.estimate(xyz, xyz, w, x, E, 4, w, x, self_pairs=False),
                 cpu.estimate(xyz, xyz, w, x, E, 4, w, x, self_pairs=False),
                 brute.zeta_brute(xyz, xyz, w, x, E, 4, w, x, self_pairs=False)):
        assert p == pairs
        assert np.abs(z - gold).max() < 1e-14
    # weighted random catalogue: the C oracle's removal equals the NumPy one
    xyz, w, x = pins.random_cap(400, 3.0, 17)
    E = pins.small_edges(5)
    zc, pc = cpu.estimate(xyz, xyz, w, x, E, 4, w, x, self_pairs=False)
    zr, pr = ref.estimate(xyz, xyz, w, x, E, 4, w, x, self_pairs=False)
    assert pc == pr
    assert pins.rel_err(zc, zr) < 1e-12


@pytest.mark.parametrize("n", [50, 120, 500])
def test_p1_brute_sizes(n):
    pins.check_brute(n=n, seed=100 + n, m_max=3)


def test_p1_brute_cap20k_subset():
    """Brute-force triplets on the first 2,000 points of the cap catalogue (cap20k workload)."""
    from synth import CONFIGS, make_positions, make_values
    cfg = CONFIGS["cap20k"]
    xyz_t = make_positions(cfg)
    x = make_values(cfg, xyz_t).numpy()[:2000]
    xyz = xyz_t.numpy()[:, :2000]
    w = np.ones(2000)
    E = cfg.edges_chord2()
    z, pairs = ref.estimate(xyz, xyz, w, x, E, cfg.m_max, w, x)
    zb, pb = brute.zeta_brute(xyz, xyz, w, x, E, cfg.m_max, w, x)
    assert pairs == pb
    for m in range(cfg.m_max + 1):
        assert pins.rel_err(z[m], zb[m]) <= 1e-12


def test_p3_hermitian_exact():
    xyz, w, x = pins.random_cap(300, 3.0, 4)
    E = pins.small_edges(6)
    for z in (ref.estimate(xyz, xyz, w, x, E, 5, w, x)[0], cpu.estimate(xyz, xyz, w, x, E, 5, w, x)[0]):
        assert np.array_equal(z, np.conj(np.swapaxes(z, 1, 2)))
        assert np.all(np.diagonal(z, axis1=1, axis2=2).imag == 0.0)
        assert np.all(z[0].imag == 0.0)


def test_p4_field_scaling_exact():
    xyz, w, x = pins.random_cap(250, 3.0, 5)
    E = pins.small_edges(5)
    z1, _ = ref.estimate(xyz, xyz, w, x, E, 4, w, x)
    zm, _ = ref.estimate(xyz, xyz, w, -x, E, 4, w, -x)
    z2, _ = ref.estimate(xyz, xyz, w, 2.0 * x, E, 4, w, 2.0 * x)
    assert np.array_equal(zm, -z1)
    assert np.array_equal(z2, 8.0 * z1)
    pins.check_weight_invariance()


def test_p5_reference_direction_invariance(monkeypatch):
    xyz, w, x = pins.random_cap(300, 3.0, 6)
    E = pins.small_edges(6)
    z0, _ = ref.estimate(xyz, xyz, w, x, E, 6, w, x)
    a0, _, _ = ref.multipoles(xyz, xyz, w, x, E, 6)
    orig = ref.bearing_basis
    alpha = np.random.default_rng(0).uniform(0, 2 * np.pi, xyz.shape[1])

    def rotated(piv):
        e_n, e_e = orig(piv)
        al = alpha[: piv.shape[1]] if piv.shape[1] == len(alpha) else alpha[0]
        return np.cos(al) * e_n + np.sin(al) * e_e, -np.sin(al) * e_n + np.cos(al) * e_e

    monkeypatch.setattr(ref, "bearing_basis", rotated)
    z1, _ = ref.estimate(xyz, xyz, w, x, E, 6, w, x)
    a1, _, _ = ref.multipoles(xyz, xyz, w, x, E, 6)
    # X_m picks up a per-pivot phase, zeta does not (paper, after eq. zetamEst2)
    assert np.abs(a1 - a0).max() > 1e-3
    for m in range(7):
        assert pins.rel_err(z1[m], z0[m]) < 1e-13


def _rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


def test_p6_global_rotation_and_mirror():
    xyz, w, x = pins.random_cap(300, 3.0, 8)
    E = pins.small_edges(6)
    a, W, N = ref.multipoles(xyz, xyz, w, x, E, 5)
    z0 = ref.contract(ref.normalise(a, W), w * x) / w.sum()
    R = _rotation(3)
    xr = R @ xyz
    xr /= np.linalg.norm(xr, axis=0)
    ar, Wr, Nr = ref.multipoles(xr, xr, w, x, E, 5)
    mirror = xyz * np.array([1.0, -1.0, 1.0])[:, None]
    am, Wm, Nm = ref.multipoles(mirror, mirror, w, x, E, 5)
    for other, Wo, No, sign in ((ar, Wr, Nr, 1.0), (am, Wm, Nm, -1.0)):
        if not np.array_equal(No, N):
            pytest.skip("a near-edge pair flipped bins under the transformation")
        zo = ref.contract(ref.normalise(other, Wo), w * x) / w.sum()
        for m in range(6):
            assert pins.rel_err(zo[m].real, z0[m].real) < 1e-10
            assert pins.rel_err(zo[m].imag, sign * z0[m].imag) < 1e-10


def test_p8_m0_annulus_means():
    pins.check_m0_annulus_means()


def test_p9_resum_dirichlet():
    xyz, w, x = pins.random_cap(150, 3.0, 9)
    E = pins.small_edges(4)
    M = 5
    z, _ = ref.estimate(xyz, xyz, w, x, E, M, w, x)
    phi = np.linspace(-math.pi, math.pi, 13)
    got = ref.resum(z, phi)
    exp = brute.dirichlet_resum_brute(xyz, xyz, w, x, E, M, w, x, phi)
    assert pins.rel_err(got, exp) < 1e-12


def test_p10_pair_counts_bruteforce_loops():
    xyz, w, x = pins.random_cap(120, 3.0, 10)
    E = pins.small_edges(5)
    _, _, N = ref.multipoles(xyz, xyz, w, x, E, 0)
    _, _, Nc = cpu.multipoles(xyz, xyz, w, x, E, 0)
    nb = len(E) - 1
    cnt = np.zeros_like(N)
    for p in range(xyz.shape[1]):
        for j in range(xyz.shape[1]):
            dx, dy, dz = (float(xyz[k, j]) - float(xyz[k, p]) for k in range(3))
            d2 = (dx * dx + dy * dy) + dz * dz
            for b in range(nb):
                if E[b] <= d2 < E[b + 1]:
                    cnt[p, b] += 1
    assert np.array_equal(N, cnt)
    assert np.array_equal(Nc, cnt)


def test_p10_edge_ties_half_open():
    """A pair exactly on an edge goes to the upper bin; one exactly at E_nb is dropped."""
    xyz, w, x = pins.random_cap(60, 2.0, 12)
    d = xyz[:, 1] - xyz[:, 0]
    d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    E = np.array([d2 / 4, d2, 2 * d2])
    _, _, N = ref.multipoles(xyz[:, :1], xyz[:, :2], w[:2], x[:2], E, 0)
    assert N[0].tolist() == [0, 1]
    E2 = np.array([d2 / 4, d2 / 2, d2])
    _, _, N2 = ref.multipoles(xyz[:, :1], xyz[:, :2], w[:2], x[:2], E2, 0)
    _, _, N2c = cpu.multipoles(xyz[:, :1], xyz[:, :2], w[:2], x[:2], E2, 0)
    assert N2[0].tolist() == [0, 0] and N2c[0].tolist() == [0, 0]


def test_healpix_pair_count_matches_annulus_area():
    from synth import ring_centres
    ns = 256
    xyz = ring_centres(ns).numpy()
    E = pins.small_edges(4, lo=2.0, hi=8.0)
    idx = np.random.default_rng(0).choice(xyz.shape[1], 64, replace=False)
    _, _, N = cpu.multipoles(xyz[:, idx], xyz, np.ones(xyz.shape[1]), np.ones(xyz.shape[1]), E, 0)
    th = 2 * np.arcsin(np.sqrt(E) / 2)
    area = 2 * np.pi * (np.cos(th[:-1]) - np.cos(th[1:]))
    expected = area / (4 * np.pi / xyz.shape[1])
    assert np.all(np.abs(N.mean(0) / expected - 1) < 0.015)


def test_c_oracle_matches_reference():
    xyz, w, x = pins.random_cap(2000, 4.0, 13)
    E = pins.small_edges(8, lo=0.1, hi=2.0, log=True)
    a1, W1, N1 = ref.multipoles(xyz, xyz, w, x, E, 7)
    a2, W2, N2, isum, ihash = cpu.multipoles(xyz, xyz, w, x, E, 7, ids=True)
    assert np.array_equal(N1, N2)
    assert pins.rel_err(W2, W1) < 1e-14
    assert pins.rel_err(a2, a1) < 1e-12
    # neighbour-index sums against a direct recount
    b = ref.bin_index(ref.pair_d2(xyz[:, :5], xyz), E)
    for p in range(5):
        for k in range(len(E) - 1):
            js = np.nonzero(b[p] == k)[0].astype(np.uint64)
            assert isum[p, k] == js.sum()
            assert ihash[p, k] == cpu.mix64(js).sum(dtype=np.uint64)
    z1, p1 = ref.estimate(xyz, xyz, w, x, E, 7, w, x)
    z2, p2 = cpu.estimate(xyz, xyz, w, x, E, 7, w, x)
    assert p1 == p2
    for m in range(8):
        assert pins.rel_err(z2[m], z1[m]) < 1e-12


def test_p11_gaussian_field_zero_mean():
    """The ensemble 3PCF of a Gaussian field vanishes: seed-averaged zeta is ~0."""
    from synth.fields import gaussian_field
    import torch
    xyz, w, _ = pins.random_cap(1500, 6.0, 14)
    w = np.ones_like(w)
    E = pins.small_edges(4, lo=0.3, hi=3.0)
    zs = []
    for seed in range(16):
        g = gaussian_field(torch.from_numpy(xyz), 64, 20.0, 200.0, seed).numpy()
        zs.append(cpu.estimate(xyz, xyz, w, g, E, 3, w, g)[0])
    zs = np.array(zs)
    mean = zs.mean(0)
    se = zs.std(0, ddof=1) / math.sqrt(len(zs))
    t = np.concatenate([(mean.real / np.where(se.real > 0, se.real, 1)).ravel(),
                        (mean.imag / np.where(se.imag > 0, se.imag, 1)).ravel()])
    t = t[np.isfinite(t)]
    assert np.mean(t * t) < 3.0
    assert np.percentile(np.abs(t), 95) < 3.5
