"""GPU parity of the multi-field estimator (z3_estimate_cross).

Three fields on one set of positions (attached maps A, B, C): the pivot carries A, the bin
b1 field B and the bin b2 field C, optionally summed over the cyclic permutations (the
remark after eq. ubEstimator).  Against the FP64 oracle (per-field C-oracle multipoles and
the cross contraction, pinned by the multi-field triplet sum): pair counts exact, zeta_m
within 1e-10 (FP64 path) and 1e-6 (mixed path) per-m max-normalised error.
"""

import ctypes

import numpy as np
import pytest
import torch

import paper_2408_16847_amd as z3
from paper_2408_16847_amd import _lib
from oracle import cpu
from synth import CONFIGS, make_positions, make_values
from tests import gpu_helpers as G
from tests import pins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cap3():
    # three correlated lognormal fields on the cap20k positions (e.g. redshift bins of one sky)
    cfg = CONFIGS["cap20k"]
    xyz_t = make_positions(cfg)
    x0, x1, x2 = (make_values(cfg, xyz_t, seed=s).numpy() for s in range(3))
    fields = np.stack([x0, x0 + 0.5 * x1, x0 - 0.3 * x2])
    return cfg, xyz_t.numpy(), fields


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
@pytest.mark.parametrize("cyclic", [False, True])
def test_cap20k_cross_fields(cap3, prec, tol, cyclic):
    cfg, xyz, f = cap3
    G.say("case: cap20k three fields", prec, "cyclic" if cyclic else "single term")
    E = cfg.edges_chord2()
    w = np.ones(xyz.shape[1])
    idx = G.build(xyz, f, E)
    z, pairs = z3.estimate_cross(idx, (0, 1, 2), cfg.m_max, prec=prec, cyclic=cyclic)
    zo, po = cpu.estimate_cross(xyz, xyz, w, tuple(f), E, cfg.m_max, w, tuple(f), cyclic=cyclic)
    assert pairs == po
    e = G.err_m(z, zo)
    G.say("err_m", prec, e)
    assert e.max() <= tol, e


def test_cross_of_one_field_is_the_estimator(cap3):
    cfg, xyz, f = cap3
    G.say("case: cross of one field")
    E = cfg.edges_chord2()
    idx = G.build(xyz, f, E)
    z, pairs = z3.estimate(idx, cfg.m_max, map_index=1)
    z1, p1 = z3.estimate_cross(idx, (1, 1, 1), cfg.m_max)
    z3c, p3 = z3.estimate_cross(idx, (1, 1, 1), cfg.m_max, cyclic=True)
    assert pairs == p1 == p3
    assert G.err_m(z1, z).max() < 1e-12
    assert G.err_m(z3c, 3.0 * z).max() < 1e-12
    # exchanging the two neighbour fields conjugates and transposes
    zbc, _ = z3.estimate_cross(idx, (0, 1, 2), cfg.m_max)
    zcb, _ = z3.estimate_cross(idx, (0, 2, 1), cfg.m_max)
    assert G.err_m(zcb, np.conj(np.swapaxes(zbc, 1, 2))).max() < 1e-12


# weighted fields, two of them white noise (zeta a sum of terms of random sign, condition
# number ~ sqrt(pivots)), both precisions
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_weighted_cross_fields_and_pivot_ranges(prec, tol):
    G.say("case: weighted cap three fields", prec)
    xyz, w, xa = pins.random_cap(3000, 4.0, 41)
    rng = np.random.default_rng(42)
    f = np.stack([xa, xa + rng.normal(size=3000), rng.normal(size=3000)])
    E = pins.small_edges(6, lo=0.05, hi=1.5, log=True)
    idx = G.build(xyz, f, E, w=w)
    zo, po = cpu.estimate_cross(xyz, xyz, w, tuple(f), E, 5, w, tuple(f), cyclic=True)
    zr = torch.zeros((6, 6, 6, 2), dtype=torch.float64, device="cuda")
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    pt = torch.zeros(1, dtype=torch.int64, device="cuda")
    for p0, p1 in ((0, 333), (333, 2100), (2100, 3000)):
        z3.estimate_cross_raw(idx, (0, 1, 2), 5, prec, True, p0, p1, zeta=zr, pair_total=pt, sum_w=sw)
    torch.cuda.synchronize()
    zc = zr.cpu().numpy() / sw.item()
    assert int(pt.item()) == po
    assert G.err_m(zc[..., 0] + 1j * zc[..., 1], zo).max() <= tol


# many bins: the contraction's wider tile shapes (2 nb = 60, 80, 128 rows: 4 x 4 tile pairs
# in one block, 5 x 5 and 8 x 8 in groups of 16 pairs per block)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
@pytest.mark.parametrize("nbins", [30, 40, 64])
def test_cross_fields_many_bins(prec, tol, nbins):
    G.say("case: three fields,", nbins, "bins", prec)
    xyz, w, xa = pins.random_cap(2500, 5.0, 43)
    rng = np.random.default_rng(44)
    f = np.stack([xa, xa + 0.5 * rng.normal(size=2500), xa - 0.3 * rng.normal(size=2500)])
    E = pins.small_edges(nbins, lo=0.05, hi=2.0, log=True)
    idx = G.build(xyz, f, E, w=w)
    z, pairs = z3.estimate_cross(idx, (0, 1, 2), 4, prec=prec, cyclic=True)
    zo, po = cpu.estimate_cross(xyz, xyz, w, tuple(f), E, 4, w, tuple(f), cyclic=True)
    assert pairs == po
    e = G.err_m(z, zo)
    G.say("err_m", prec, e)
    assert e.max() <= tol, e


def test_cross_rejects_a_missing_map():
    G.say("case: z3_estimate_cross map range")
    xyz, E, x = pins.three_point_case()
    idx = G.build(xyz, np.stack([x, x]), E)
    zeta = torch.zeros((5, 3, 3, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.Zeta3Error) as ei:
        _lib.call("z3_estimate_cross", idx.handle, 0, 1, 2, 0, 4, 0, 0, 3, ctypes.c_void_p(zeta.data_ptr()),
                  ctypes.c_void_p(0), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert ei.value.status == 1
    torch.cuda.synchronize()
    assert torch.count_nonzero(zeta).item() == 0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_cross_fields_in_different_map_groups(cap3, prec, tol):
    # maps 0, 4 and 5 of six attached maps: not one group of four, so each field's
    # multipoles come from its own one-map pass (maps 0, 1, 2 share one many-map pass)
    cfg, xyz, f = cap3
    G.say("case: cap20k fields in different map groups", prec)
    E = cfg.edges_chord2()
    w = np.ones(xyz.shape[1])
    six = np.concatenate([f, f[::-1]])  # maps 3, 4, 5 = fields 2, 1, 0
    idx = G.build(xyz, six, E)
    z, pairs = z3.estimate_cross(idx, (0, 4, 5), cfg.m_max, prec=prec, cyclic=True)
    fo = (f[0], f[1], f[0])
    zo, po = cpu.estimate_cross(xyz, xyz, w, fo, E, cfg.m_max, w, fo, cyclic=True)
    assert pairs == po
    assert G.err_m(z, zo).max() <= tol
    zg, pg = z3.estimate_cross(idx, (0, 1, 0), cfg.m_max, prec=prec, cyclic=True)
    assert pg == pairs
    assert G.err_m(zg, zo).max() <= tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_cross_fields_in_the_last_slot_of_a_group(cap3, prec, tol):
    # four attached maps, fields read from slots 1, 2, 3 and 3, 0, 2 of the group: the shared
    # pass then carries all four maps per lane, where fields 0, 1, 2 need only three
    cfg, xyz, f = cap3
    G.say("case: cap20k fields in slot 3 of a map group", prec)
    E = cfg.edges_chord2()
    w = np.ones(xyz.shape[1])
    four = np.concatenate([f, (f[1] - f[2])[None]])
    idx = G.build(xyz, four, E)
    for maps in ((1, 2, 3), (3, 0, 2)):
        z, pairs = z3.estimate_cross(idx, maps, cfg.m_max, prec=prec, cyclic=True)
        fo = tuple(four[k] for k in maps)
        zo, po = cpu.estimate_cross(xyz, xyz, w, fo, E, cfg.m_max, w, fo, cyclic=True)
        assert pairs == po
        e = G.err_m(z, zo)
        G.say("err_m", maps, prec, e.max())
        assert e.max() <= tol


def _catalogues():
    # three different point sets on one 4-degree cap, each with its own weights and a
    # lognormal field (galaxy samples of different surveys, say)
    from synth import lognormal_field
    out = []
    for k, n in enumerate((2500, 3200, 2800)):
        xyz, w, _ = pins.random_cap(n, 4.0, 301 + k)
        x = lognormal_field(torch.from_numpy(xyz), 64, 20.0, 200.0, 11 + k).numpy()
        out.append((xyz, w, x))
    return out


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_cross_distinct_catalogues(prec, tol):
    from oracle import ref
    G.say("case: three distinct catalogues", prec)
    cats = _catalogues()
    E = pins.small_edges(6, lo=0.05, hi=1.2, log=True)
    idxs = [G.build(xyz, x, E, w=w) for xyz, w, x in cats]
    total = 0
    total_o = 0
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        pa, wa, xa = cats[a]
        sw = torch.zeros(1, dtype=torch.float64, device="cuda")
        zt, pb, pc = z3.estimate_cross_catalogues(idxs[b], idxs[c], torch.from_numpy(pa).cuda(),
                                                  torch.from_numpy(xa).cuda(), torch.from_numpy(wa).cuda(), 5,
                                                  prec=prec, sum_w=sw)
        torch.cuda.synchronize()
        zg = zt.cpu().numpy() / sw.item()
        zg = zg[..., 0] + 1j * zg[..., 1]
        zo, pbo, pco = ref.estimate_cross_catalogues(pa, wa, xa, *cats[b], *cats[c], E, 5)
        assert (pb, pc) == (pbo, pco)
        assert G.err_m(zg, zo).max() <= tol
        total = total + zg
        total_o = total_o + zo
    assert G.err_m(total, total_o).max() <= tol


def test_cross_catalogues_one_catalogue_and_bad_bins():
    G.say("case: distinct-catalogue entry, one catalogue, mismatched bins")
    xyz, w, x = _catalogues()[0]
    E = pins.small_edges(6, lo=0.05, hi=1.2, log=True)
    idx = G.build(xyz, x, E, w=w)
    z, pairs = z3.estimate(idx, 5)
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    zt, pb, pc = z3.estimate_cross_catalogues(idx, idx, torch.from_numpy(xyz).cuda(), torch.from_numpy(x).cuda(),
                                              torch.from_numpy(w).cuda(), 5, sum_w=sw)
    torch.cuda.synchronize()
    zg = zt.cpu().numpy() / sw.item()
    assert pb == pc == pairs
    assert G.err_m(zg[..., 0] + 1j * zg[..., 1], z).max() < 1e-12
    idx2 = G.build(xyz, x, pins.small_edges(6, lo=0.05, hi=1.3, log=True), w=w)
    with pytest.raises(_lib.Zeta3Error) as ei:
        z3.estimate_cross_catalogues(idx, idx2, torch.from_numpy(xyz).cuda(), torch.from_numpy(x).cuda(), None, 5)
    assert ei.value.status == 1
