"""GPU many-map estimator: the MFMA kernel (more than 4 maps) and the register-tiled kernel
(up to 4 maps) against the oracle, every map tile against the others (bit-identical), and
against the one-map kernel."""

import math

import numpy as np
import pytest
import torch

import paper_2408_16847_amd as z3
from oracle import cpu
from synth import CONFIGS, make_values, ring_centres
from synth.bins import chord2_edges, theta_edges
from tests import gpu_helpers as G
from tests import pins

pytestmark = pytest.mark.gpu

SHAPES = [(4, 16), (2, 32), (2, 16), (4, 32)]  # (waves per block, maps per wave)


def _raw(idx, M, prec, p0=0, p1=None):
    zeta = torch.zeros((idx.nmaps, M + 1, idx.nbins, idx.nbins, 2), dtype=torch.float64, device="cuda")
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    z3.estimate_maps_raw(idx, M, prec, p0, p1, zeta, pairs)
    torch.cuda.synchronize()
    return zeta.cpu().numpy(), int(pairs.item())


def _lognormal_maps(xyz, nmaps):
    """Lognormal fields of the 10-degree-cap recipe, one seed per map."""
    xyz_t = torch.from_numpy(np.ascontiguousarray(xyz))
    return np.stack([make_values(CONFIGS["cap20k"], xyz_t, seed=s).numpy() for s in range(nmaps)])


@pytest.fixture(scope="module")
def weighted_cap64():
    xyz, w, _ = pins.random_cap(3000, 5.0, 23)
    xs = _lognormal_maps(xyz, 64)
    E = pins.small_edges(6, lo=0.05, hi=2.5, log=True)
    return xyz, w, xs, E


# Lognormal maps (the estimator's workload) and white-noise maps (zero mean, no correlation:
# zeta is a sum of terms of random sign, condition number sum |t| / |sum t| ~ sqrt(pivots)
# ~ 55 here), both precisions.
@pytest.mark.parametrize("field,prec,tol", [("lognormal", "fp64", 1e-10), ("lognormal", "mixed", 1e-6),
                                            ("white", "fp64", 1e-10), ("white", "mixed", 1e-6)])
def test_batch_tiles_identical_and_match_oracle(weighted_cap64, field, prec, tol):
    G.say("case: batch tiles", field, prec)
    xyz, w, xs, E = weighted_cap64
    if field == "white":
        xs = np.random.default_rng(8).normal(size=xs.shape)
    M = 8
    idx = G.build(xyz, xs, E, w=w)
    outs = {}
    for shape in SHAPES:
        idx.set_batch_shape(*shape)
        assert idx.batch_shape(M, prec) == shape
        outs[shape] = _raw(idx, M, prec)
        G.say("shape", shape, "pairs", outs[shape][1])
    ref = outs[SHAPES[0]]
    for shape in SHAPES[1:]:
        assert outs[shape][1] == ref[1]
        assert np.array_equal(outs[shape][0], ref[0]), shape
    sw = w.sum()
    z = ref[0] / sw
    for s in (0, 17, 63):
        zo, po = cpu.estimate(xyz, xyz, w, xs[s], E, M, w, xs[s])
        assert po == ref[1]
        e = G.err_m(z[s, ..., 0] + 1j * z[s, ..., 1], zo)
        z1, _ = z3.estimate(idx, M, prec=prec, map_index=s)
        e1 = G.err_m(z1, zo)
        G.say("map", s, "err", e.max(), "one-map kernel err", e1.max())
        assert e.max() < tol, (s, e)
        assert e1.max() < tol, (s, e1)
    idx.free()


def test_batch_autotune_picks_a_shape(weighted_cap64):
    G.say("case: batch autotune")
    xyz, w, xs, E = weighted_cap64
    idx = G.build(xyz, xs, E, w=w)  # 64 maps: the MFMA kernel on both paths
    assert idx.batch_shape(6, "fp64") == (0, 0)
    a, pa = _raw(idx, 6, "fp64")
    t = idx.batch_shape(6, "fp64")
    G.say("tuned shape", t)
    assert t in SHAPES
    idx.set_batch_shape(2, 16)
    b, pb = _raw(idx, 6, "fp64")
    assert pa == pb and np.array_equal(a, b)
    idx.set_batch_shape(0, 0)
    idx.set_values(torch.from_numpy(xs).cuda())  # new values forget the tuned shape
    assert idx.batch_shape(6, "fp64") == (0, 0)
    with pytest.raises(z3.Zeta3Error):
        idx.set_batch_shape(3, 16)
    idx.free()


@pytest.mark.parametrize("nmaps", [2, 3, 4, 20, 32, 60])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_many_maps_match_one_map_kernel(nmaps, prec):
    """HEALPix Nside 64 (full sky: poles, wrap-around, full bands), maps against the FP64
    one-map kernel; 2 maps run one-map passes, 3-4 maps the register-tiled kernel, 20 maps
    that kernel group by group, 32 maps the groups on the FP64 path and the MFMA kernel on the
    mixed one, 60 maps the MFMA kernel."""
    G.say("case: many maps vs one-map kernel", nmaps, prec)
    xyz_t = ring_centres(64)
    cfg = CONFIGS["nside512"]
    xs = torch.stack([make_values(cfg, xyz_t, seed=s) for s in range(nmaps)])
    E = chord2_edges(theta_edges(math.radians(0.5), math.radians(12.0), 7, True))
    M = 10
    idx = z3.Index(xyz_t.cuda(), E)
    idx.set_values(xs.cuda())
    zs, pairs = z3.estimate_maps(idx, M, prec=prec)
    tol = 1e-12 if prec == "fp64" else 1e-6
    for s in sorted({0, nmaps // 2, nmaps - 1}):
        # the reference is the FP64 one-map kernel (itself within 1e-10 of the oracle)
        z1, p1 = z3.estimate(idx, M, prec="fp64", map_index=s)
        assert p1 == pairs
        e = G.err_m(zs[s], z1)
        G.say("map", s, "err vs one-map FP64 kernel", e.max())
        assert e.max() < tol, (s, e)
    idx.free()


@pytest.mark.parametrize("M", [0, 1, 7, 8, 15, 16])
def test_batch_harmonic_column_tiles(M):
    """m_max at the edges of the 16-column MFMA tiles (2M+1 = 1, 3, 15, 17, 31, 33 columns);
    five maps, the MFMA kernel selected by a fixed block shape."""
    G.say("case: batch column tiles, M =", M)
    xyz, w, _ = pins.random_cap(1200, 3.0, 5)
    xs = _lognormal_maps(xyz, 5)
    E = pins.small_edges(4, lo=0.1, hi=1.5, log=False)
    idx = G.build(xyz, xs, E, w=w)
    idx.set_batch_shape(4, 16)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        zs, pairs = z3.estimate_maps(idx, M, prec=prec)
        for s in (0, 4):
            zo, po = cpu.estimate(xyz, xyz, w, xs[s], E, M, w, xs[s])
            assert po == pairs
            e = G.err_m(zs[s], zo)
            assert e.max() < tol, (prec, s, e)
    idx.free()


def test_batch_pivot_subranges_compose(weighted_cap64):
    """Pivot ranges processed in pieces (ragged, not multiples of the 4-pivot block) sum
    to the whole."""
    G.say("case: batch pivot sub-ranges")
    xyz, w, xs, E = weighted_cap64
    idx = G.build(xyz, xs[:24], E, w=w)
    n = xyz.shape[1]
    whole, pw = _raw(idx, 6, "fp64")
    cuts = [0, 1, 7, 1234, 2999, n]
    acc = torch.zeros((24, 7, 6, 6, 2), dtype=torch.float64, device="cuda")
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    for a, b in zip(cuts[:-1], cuts[1:]):
        z3.estimate_maps_raw(idx, 6, "fp64", a, b, acc, pairs)
    torch.cuda.synchronize()
    assert int(pairs.item()) == pw
    part = acc.cpu().numpy()
    assert np.abs(part - whole).max() <= 1e-12 * np.abs(whole).max()
    idx.free()


@pytest.mark.parametrize("nb,M", [(20, 10), (25, 8)])
@pytest.mark.parametrize("nmaps,shape", [(1, None), (3, None), (6, None), (6, (2, 16))])
def test_contraction_unit_budgets(nb, M, nmaps, shape):
    """The contraction at both sides of its register budget: 20 bins with m <= 10 (66
    (m, tile pair) units, the LDS-staged kernel at 9 units per wave) and 25 bins with m <= 8
    (90 units, beyond it: the tile-pair kernel, after a transpose on the many-map path), for
    the one-map kernel, the register-tiled kernel (3 maps; 6 maps in two groups) and the MFMA
    kernel (6 maps with a fixed block shape)."""
    G.say("case: contraction units, nb", nb, "M", M, "maps", nmaps, "shape", shape)
    xyz, w, _ = pins.random_cap(1500, 4.0, 11)
    xs = _lognormal_maps(xyz, nmaps)
    E = pins.small_edges(nb, lo=0.05, hi=2.0, log=True)
    idx = G.build(xyz, xs if nmaps > 1 else xs[0], E, w=w)
    if shape:
        idx.set_batch_shape(*shape)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        zs, pairs = z3.estimate_maps(idx, M, prec=prec)
        for s in sorted({0, nmaps - 1}):
            zo, po = cpu.estimate(xyz, xyz, w, xs[s], E, M, w, xs[s])
            assert po == pairs
            e = G.err_m(zs[s], zo)
            G.say("  map", s, prec, "err", e.max())
            assert e.max() < tol, (prec, s, e)
    idx.free()
