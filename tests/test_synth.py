"""Input generators: HEALPix RING geometry, cap sampler, lognormal field, bin edges."""

import math

import numpy as np
import torch

from synth import CONFIGS, cap_points, chord2_edges, degrade_ring, npix, ring_centres, theta_edges
from synth.fields import field_params, lognormal_field
from synth.healpix import ang2pix_ring


def test_healpix_counts_rings_and_norms():
    for ns in (1, 2, 4, 16, 64):
        xyz, ring, z, omz, phi = ring_centres(ns, with_ring=True)
        assert xyz.shape == (3, npix(ns))
        counts = torch.bincount(ring).numpy()
        assert len(counts) == 4 * ns - 1
        i = np.arange(1, 4 * ns)
        exp = np.where(i < ns, 4 * i, np.where(i > 3 * ns, 4 * (4 * ns - i), 4 * ns))
        assert np.array_equal(counts, exp)
        assert float(((xyz * xyz).sum(0) - 1).abs().max()) < 1e-15
        zr = np.full(4 * ns - 1, -np.inf)
        np.maximum.at(zr, ring.numpy(), z.numpy())
        assert np.abs(zr + zr[::-1]).max() <= 1e-15
        assert float(phi.min()) >= 0 and float(phi.max()) < 2 * math.pi


def test_healpix_point_to_pixel_inverts_centres():
    for ns in (1, 2, 8, 32):
        _, _, z, omz, phi = ring_centres(ns, with_ring=True)
        assert torch.equal(ang2pix_ring(ns, z, omz, phi), torch.arange(npix(ns)))


def test_healpix_nearest_neighbour_spacing():
    ns = 32
    xyz = ring_centres(ns).numpy()
    idx = np.random.default_rng(0).choice(xyz.shape[1], 200, replace=False)
    d = np.arccos(np.clip(xyz[:, idx].T @ xyz, -1, 1))
    d[np.arange(200), idx] = np.inf
    nn = d.min(1).mean()
    assert 0.8 < nn / math.sqrt(4 * math.pi / npix(ns)) < 1.2


def test_degrade_keeps_four_children():
    v = torch.randn(npix(16), dtype=torch.float64)
    pos, vm, ws = degrade_ring(16, v)
    assert pos.shape == (3, npix(8))
    assert torch.all(ws == 4.0)
    assert abs(float(vm.sum() * 4 - v.sum())) < 1e-9


def test_cap_points_inside_cap():
    xyz = cap_points(5000, 10.0, seed=3).numpy()
    assert np.all(xyz[0] >= math.cos(math.radians(10.0)) - 1e-15)
    assert np.abs((xyz * xyz).sum(0) - 1).max() < 1e-15


def test_lognormal_mean_zero_and_rounding():
    amp, *_ , var_g = field_params(256, 20, 800, 0)
    assert abs(var_g - 0.5 * np.sum(amp ** 2)) < 1e-15
    xyz = ring_centres(32)
    d = lognormal_field(xyz, 64, 20.0, 200.0, 1)
    assert float(d.min()) > -1.0
    d32 = lognormal_field(xyz, 64, 20.0, 200.0, 1, fp32_values=True)
    assert torch.equal(d32, d32.float().double())


def test_bin_edges():
    e = theta_edges(1.0, 8.0, 3, True)
    assert np.allclose(e, [1, 2, 4, 8])
    e = theta_edges(1.0, 4.0, 3, False)
    assert np.allclose(e, [1, 2, 3, 4])
    c = chord2_edges(np.array([math.pi / 3]))
    assert abs(c[0] - 1.0) < 1e-15
    for cfg in CONFIGS.values():
        E = cfg.edges_chord2()
        assert len(E) == cfg.nbins + 1 and np.all(np.diff(E) > 0) and E[0] > 0
