"""GPU parity at the full workload sizes the bench times (HEALPix Nside 2048 and 4096, the
approximate Nside 4096 search, 64 maps at Nside 512, Nside 2048 without the k = j terms,
the flat plane3m map), on sampled pivots the oracle computes
one by one: ragged pivot ranges
at the north pole, across a band boundary near the equator (the 0 / 2 pi wrap of the
longitude windows) and at the south pole.  Per-pivot pair counts, bin weights and neighbour
fingerprints bit-exact; per-pivot multipoles within 1e-11 (FP64) of each bin's scale, and
within 1.2e-7 on the mixed path (its multipoles are FP64 sums rounded once to FP32, an error
of at most 2^-24 of each value); zeta over all sampled pivots within 1e-10 / 1e-6, with and
without the k = j terms, each against its own per-m maximum."""

import numpy as np
import pytest
import torch

import paper_2408_16847_amd as z3
from oracle import cpu
from synth import CONFIGS, make_positions, make_values
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


def _ranges(xyz_h, perm):
    """Ragged pivot ranges in index order (latitude bands from the north pole, longitude
    cells within a band): the first band(s), a range across a band boundary near the
    equator (the end of one band at phi near 2 pi, the start of the next at phi near 0),
    and the last band(s)."""
    n = len(perm)
    lo = max(n // 2 - 20000, 0)
    seg = perm[lo:n // 2 + 20000]
    phi = np.arctan2(xyz_h[1, seg], xyz_h[0, seg]) % (2 * np.pi)
    jumps = np.nonzero(phi[1:] < phi[:-1] - np.pi)[0]
    wrap = lo + int(jumps[0]) + 1 if len(jumps) else n // 2
    return [(0, 397), (wrap - 150, wrap + 251), (n - 430, n)]


def _check_multipoles(idx, xyz_h, x_h, E, M, p0, p1, perm):
    pm = perm[p0:p1]
    w = np.ones(xyz_h.shape[1])
    ao, Wo, No, _, Ho = cpu.multipoles(xyz_h[:, pm], xyz_h, w, x_h, E, M, ids=True)
    scale = np.abs(ao).max(axis=1, keepdims=True) + 1e-300
    for prec, tol in (("fp64", 1e-11), ("mixed", 1.2e-7)):
        a, W, N, H = G.gpu_multipoles(idx, M, p0, p1, prec=prec, norm="none")
        assert np.array_equal(N, No), prec
        assert np.array_equal(W, Wo), prec
        assert np.array_equal(H, Ho), prec
        err = (np.abs(a - ao) / scale).max()
        G.say("  multipoles", prec, "pivots", p0, p1, "err", err)
        assert err < tol, (prec, err)


def _check_zeta(idx, xyz_h, x_h, E, M, ranges, perm, self_pairs=True):
    pm = np.concatenate([perm[p0:p1] for p0, p1 in ranges])
    w = np.ones(xyz_h.shape[1])
    zo, po = cpu.estimate(xyz_h[:, pm], xyz_h, w, x_h, E, M, np.ones(len(pm)), x_h[pm], self_pairs=self_pairs)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        zeta = torch.zeros((M + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
        pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        for p0, p1 in ranges:
            z3.estimate_raw(idx, M, prec, p0, p1, zeta=zeta, pair_total=pairs, self_pairs=self_pairs)
        torch.cuda.synchronize()
        zg = zeta.cpu().numpy() / len(pm)
        zg = zg[..., 0] + 1j * zg[..., 1]
        assert int(pairs.item()) == po
        e = G.err_m(zg, zo).max()
        G.say("  zeta", prec, "self pairs" if self_pairs else "no self pairs", len(pm), "pivots, err", e)
        assert e < tol, (prec, e)


@pytest.mark.parametrize("name", ["nside2048", "nside4096"])
def test_fullsize_healpix_sampled_pivots(name):
    cfg = CONFIGS[name]
    G.say("case: full size", name)
    xyz = make_positions(cfg, device="cuda")
    x = make_values(cfg, xyz, seed=0)
    E = cfg.edges_chord2()
    idx = z3.Index(xyz, E)
    idx.set_values(x)
    perm = idx.perm().cpu().numpy()
    xyz_h, x_h = xyz.cpu().numpy(), x.cpu().numpy()
    del xyz
    ranges = _ranges(xyz_h, perm)
    for p0, p1 in ranges:
        _check_multipoles(idx, xyz_h, x_h, E, cfg.m_max, p0, p1, perm)
    _check_zeta(idx, xyz_h, x_h, E, cfg.m_max, ranges, perm)
    if name == "nside2048":
        _check_zeta(idx, xyz_h, x_h, E, cfg.m_max, ranges, perm, self_pairs=False)
    idx.free()


def test_fullsize_plane3m_sampled_pivots():
    """The flat workload (1774 x 1774 jittered grid, 15 log bins 1-40 units, m <= 10):
    ragged pivot ranges at the first strips, the middle and the last strips, against the
    planar oracle over all 3.1e6 neighbours."""
    from oracle import ref
    cfg = CONFIGS["plane3m"]
    G.say("case: full size plane3m")
    xy = make_positions(cfg, device="cuda")
    x = make_values(cfg, xy, seed=0)
    E = cfg.edges_chord2()
    idx = z3.Index(xy, E, planar=True)
    idx.set_values(x)
    perm = idx.perm().cpu().numpy()
    xy_h, x_h = xy.cpu().numpy(), x.cpu().numpy()
    n = len(perm)
    ranges = [(0, 150), (n // 2 - 77, n // 2 + 123), (n - 170, n)]
    w = np.ones(n)
    M = cfg.m_max
    rmax = np.sqrt(E[-1]) * (1 + 1e-6) + 1e-9

    def near(piv_idx):
        # neighbours inside the pivots' bounding box grown by the largest radius: every point
        # outside it is farther than the last edge from every pivot, so the oracle's sums
        # over this subset equal those over the whole map
        lo = xy_h[:, piv_idx].min(1) - rmax
        hi = xy_h[:, piv_idx].max(1) + rmax
        return np.nonzero(np.all((xy_h >= lo[:, None]) & (xy_h <= hi[:, None]), axis=0))[0]

    for p0, p1 in ranges:
        sel = near(perm[p0:p1])
        ao, Wo, No = ref.multipoles_planar(xy_h[:, perm[p0:p1]], xy_h[:, sel], w[sel], x_h[sel], E, M)
        scale = np.abs(ao).max(axis=1, keepdims=True) + 1e-300
        for prec, tol in (("fp64", 1e-11), ("mixed", 1.2e-7)):
            out = z3.accumulate(idx, M, p0, p1, prec=prec, norm="none", want_w=True, want_counts=True)
            A = out["A"].double().cpu().numpy()
            a = np.transpose(A[:, 0] + 1j * A[:, 1], (2, 0, 1))
            assert np.array_equal(out["counts"].cpu().numpy().T, No), prec
            assert np.array_equal(out["W"].cpu().numpy().T, Wo), prec
            err = (np.abs(a - ao) / scale).max()
            G.say("  plane multipoles", prec, p0, p1, "err", err)
            assert err < tol, (prec, err)
    pm = np.concatenate([perm[p0:p1] for p0, p1 in ranges])
    sel = np.unique(np.concatenate([near(perm[p0:p1]) for p0, p1 in ranges]))
    zo, po = ref.estimate_planar(xy_h[:, pm], xy_h[:, sel], w[sel], x_h[sel], E, M, np.ones(len(pm)), x_h[pm])
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        zeta = torch.zeros((M + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
        pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        for p0, p1 in ranges:
            z3.estimate_raw(idx, M, prec, p0, p1, zeta=zeta, pair_total=pairs)
        torch.cuda.synchronize()
        zg = zeta.cpu().numpy() / len(pm)
        assert int(pairs.item()) == po
        e = G.err_m(zg[..., 0] + 1j * zg[..., 1], zo).max()
        G.say("  plane zeta", prec, len(pm), "pivots, err", e)
        assert e < tol, (prec, e)
    idx.free()


def test_fullsize_batch64_sampled_pivots():
    """The MFMA many-map kernel over all 64 maps at Nside 512, on sampled pivots, for the
    first, a middle and the last map."""
    cfg = CONFIGS["batch64"]
    G.say("case: full size batch64")
    xyz = make_positions(cfg, device="cuda")
    x = torch.stack([make_values(cfg, xyz, seed=s) for s in range(cfg.nmaps)])
    E = cfg.edges_chord2()
    M = cfg.m_max
    idx = z3.Index(xyz, E)
    idx.set_values(x)
    perm = idx.perm().cpu().numpy()
    xyz_h, x_h = xyz.cpu().numpy(), x.cpu().numpy()
    w = np.ones(xyz_h.shape[1])
    ranges = _ranges(xyz_h, perm)
    pm = np.concatenate([perm[p0:p1] for p0, p1 in ranges])
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        zeta = torch.zeros((cfg.nmaps, M + 1, cfg.nbins, cfg.nbins, 2), dtype=torch.float64, device="cuda")
        pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        for p0, p1 in ranges:
            z3.estimate_maps_raw(idx, M, prec, p0, p1, zeta, pairs)
        torch.cuda.synchronize()
        zg = zeta.cpu().numpy() / len(pm)
        for s in (0, 31, 63):
            zo, po = cpu.estimate(xyz_h[:, pm], xyz_h, w, x_h[s], E, M, np.ones(len(pm)), x_h[s][pm])
            assert int(pairs.item()) == po
            e = G.err_m(zg[s, ..., 0] + 1j * zg[s, ..., 1], zo).max()
            G.say("  map", s, prec, len(pm), "pivots, err", e)
            assert e < tol, (s, prec, e)
    idx.free()


def test_fullsize_approx_nside4096_sampled_pivots():
    """The approximate search at full size: Nside 4096 pivots (external catalogue, RING
    order) against the Nside 2048 averaged neighbour map, on pivot ranges at the north pole,
    across the equator and at the south pole, against the oracle run on the same coarse
    neighbour catalogue."""
    from synth import degrade_ring
    cfg = CONFIGS["nside4096"]
    G.say("case: full size approx nside4096")
    xyz = make_positions(cfg, device="cuda")
    x = make_values(cfg, xyz, seed=0)
    nxyz, nx, nw = degrade_ring(cfg.n_or_nside, x)
    E = cfg.edges_chord2()
    M = cfg.m_max
    idx = z3.Index(nxyz, E, weights=nw)
    idx.set_values(nx)
    n = xyz.shape[1]
    ranges = [(0, 300), (n // 2 - 150, n // 2 + 151), (n - 300, n)]
    piv_h = np.concatenate([xyz[:, a:b].cpu().numpy() for a, b in ranges], axis=1)
    pxv_h = np.concatenate([x[a:b].cpu().numpy() for a, b in ranges])
    nbr_h, nx_h, nw_h = nxyz.cpu().numpy(), nx.cpu().numpy(), nw.cpu().numpy()
    zo, po = cpu.estimate(piv_h, nbr_h, nw_h, nx_h, E, M, np.ones(piv_h.shape[1]), pxv_h)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        zeta = torch.zeros((M + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
        pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        for a, b in ranges:
            z3.estimate_pivots_raw(idx, xyz, x, None, M, prec=prec, p0=a, p1=b, zeta=zeta, pair_total=pairs)
        torch.cuda.synchronize()
        zg = zeta.cpu().numpy() / piv_h.shape[1]
        assert int(pairs.item()) == po, (prec, int(pairs.item()), po)
        e = G.err_m(zg[..., 0] + 1j * zg[..., 1], zo).max()
        G.say("  approx zeta", prec, piv_h.shape[1], "pivots, err", e)
        assert e < tol, (prec, e)
    idx.free()
