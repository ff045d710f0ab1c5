"""GPU adjoint (z3_adjoint / Zeta3Fn.backward) against the oracle gradient and central
finite differences of the GPU forward."""

import math

import numpy as np
import pytest
import torch

import paper_2408_16847_amd as z3
from oracle import grad as ograd
from synth import CONFIGS, make_values, ring_centres
from synth.bins import chord2_edges, theta_edges
from tests import gpu_helpers as G
from tests import pins

pytestmark = pytest.mark.gpu


def _rand_G(seed, M, nb):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(M + 1, nb, nb)) + 1j * rng.normal(size=(M + 1, nb, nb))


def _G_tensor(Gc):
    return torch.from_numpy(np.stack([Gc.real, Gc.imag], -1)).cuda()


# 6 and 20 bins: the prep kernel's register paths (up to 16 and 32 bins); 40: its
# general path
@pytest.mark.parametrize("weighted,nb", [(False, 6), (True, 6), (False, 20), (True, 40)])
def test_adjoint_matches_oracle_gradient(weighted, nb):
    G.say("case: adjoint vs oracle, weighted", weighted, "bins", nb)
    xyz, w, x = pins.random_cap(1500, 4.0, 91)
    if not weighted:
        w = np.ones_like(w)
    E = pins.small_edges(nb, lo=0.1, hi=2.0, log=True)
    M = 6
    idx = G.build(xyz, x, E, w=w if weighted else None)
    Gc = _rand_G(5, M, nb)
    g = z3.adjoint(idx, _G_tensor(Gc), 1.0 / w.sum(), M).cpu().numpy()
    go = ograd.zeta_grad(xyz, w, x, E, M, Gc)
    err = np.abs(g - go).max() / np.abs(go).max()
    G.say("adjoint rel err", err)
    assert err < 1e-10


def test_adjoint_central_differences_of_gpu_forward():
    G.say("case: adjoint vs central differences")
    xyz_t = ring_centres(32)
    xyz = xyz_t.numpy()
    x = make_values(CONFIGS["nside512"], xyz_t).numpy()
    E = chord2_edges(theta_edges(math.radians(3.0), math.radians(20.0), 5, True))
    M = 8
    Gc = _rand_G(7, M, 5)
    idx = G.build(xyz, x, E)
    g = z3.adjoint(idx, _G_tensor(Gc), 1.0 / xyz.shape[1], M).cpu().numpy()

    def L(xx):
        idx.set_values(torch.from_numpy(xx).cuda())
        z, _ = z3.estimate(idx, M)
        return float(np.sum(Gc.real * z.real + Gc.imag * z.imag))

    for k in np.random.default_rng(3).choice(xyz.shape[1], 6, replace=False):
        h = 1.0
        xp = x.copy(); xp[k] += h
        xm = x.copy(); xm[k] -= h
        fd = (L(xp) - L(xm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-9 * max(np.abs(g).max(), 1e-300), (k, fd, g[k])


def test_autograd_quadratic_loss_batch_of_maps():
    G.say("case: autograd batch")
    xyz_t = ring_centres(16)
    cfg = CONFIGS["nside512"]
    xs = torch.stack([make_values(cfg, xyz_t, seed=s) for s in range(5)]).cuda()
    E = chord2_edges(theta_edges(math.radians(6.0), math.radians(30.0), 4, True))
    M = 6
    idx = z3.Index(xyz_t.cuda(), E)
    x = xs.clone().requires_grad_(True)
    zeta = z3.Zeta3Fn.apply(x, idx, M, "fp64")
    t = torch.from_numpy(np.random.default_rng(3).normal(size=zeta.shape)).cuda() * zeta.detach().std()
    loss = ((zeta - t) ** 2).sum()
    loss.backward()
    gx = x.grad.cpu().numpy()
    # the gradient of each map against the oracle gradient with G = 2 (zeta - t)
    for s in (0, 4):
        zc = (zeta.detach() - t)[s].cpu().numpy()
        Gc = 2.0 * (zc[..., 0] + 1j * zc[..., 1])
        go = ograd.zeta_grad(xyz_t.numpy(), np.ones(xyz_t.shape[1]), xs[s].cpu().numpy(), E, M, Gc)
        assert np.abs(gx[s] - go).max() <= 1e-10 * np.abs(go).max()


@pytest.mark.parametrize("nmaps,shape", [(3, None), (6, None), (6, (4, 16))])
def test_adjoint_maps_matches_per_map_adjoint(monkeypatch, nmaps, shape):
    """z3_adjoint_maps (multipoles of several maps recomputed together: the register-tiled
    kernel group by group, or the MFMA kernel when a block shape is fixed; several pivot
    chunks, a pivot sub-range) against z3_adjoint map by map."""
    G.say("case: adjoint_maps vs per-map adjoint", nmaps, shape)
    monkeypatch.setenv("Z3_WORKSPACE_MB", "1")
    xyz, w, _ = pins.random_cap(3000, 5.0, 17)
    E = pins.small_edges(6, lo=0.1, hi=2.5, log=True)
    M = 6
    rng = np.random.default_rng(4)
    xs = rng.normal(size=(nmaps, xyz.shape[1]))
    idx = G.build(xyz, xs, E, w=w)
    if shape:
        idx.set_batch_shape(*shape)
    Gs = torch.stack([_G_tensor(_rand_G(20 + k, M, 6)) for k in range(nmaps)])
    p0, p1 = 37, 2811
    got = z3.adjoint_maps(idx, Gs, 0.5, M, p0=p0, p1=p1).cpu().numpy()
    for k in range(nmaps):
        ref = z3.adjoint(idx, Gs[k], 0.5, M, map_index=k, p0=p0, p1=p1).cpu().numpy()
        err = np.abs(got[k] - ref).max() / np.abs(ref).max()
        G.say("map", k, "rel err", err)
        assert err < 1e-12
