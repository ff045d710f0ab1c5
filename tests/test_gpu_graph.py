"""Forward + adjoint captured in one HIP graph (GraphStep): every replay, with new field
values and eager work between replays, against the same computation run eagerly.  The
binding's normalised zeta (GraphStep, Zeta3Fn) is the library's z3_estimate(_maps)
followed by z3_finalize on the device, bit for bit."""

import numpy as np
import pytest
import torch

import paper_2408_16847_amd as z3
from synth import CONFIGS, make_values
from tests import gpu_helpers as G
from tests import pins

pytestmark = pytest.mark.gpu


def _maps(xyz, nmaps, seed0):
    xyz_t = torch.from_numpy(np.ascontiguousarray(xyz))
    return torch.stack([make_values(CONFIGS["cap20k"], xyz_t, seed=seed0 + s) for s in range(nmaps)])


def _finalized(idx, M, prec):
    """z3_estimate_maps (z3_estimate for one map), then z3_finalize with the pivot weight sum."""
    zeta = z3.estimate_maps_raw(idx, M, prec)
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    z3._lib.call("z3_pivot_weight_sum", idx.handle, 0, idx.n, z3.zeta3._ptr(sw), z3.zeta3._stream())
    z3._lib.call("z3_finalize", idx.nmaps, M, idx.nbins, z3.zeta3._ptr(zeta), z3.zeta3._ptr(sw),
                 z3.zeta3._stream())
    return zeta, float(sw.item())


def _eager(idx, x, M, prec, t):
    """zeta (normalised) and dL/dx for L = sum (zeta - t)^2, by the eager calls."""
    idx.set_values(x.cuda())
    zeta, s = _finalized(idx, M, prec)
    scale = 1.0 / s
    g = (2.0 * (zeta - t)).contiguous()
    if idx.nmaps > 1:
        grad = z3.adjoint_maps(idx, g, scale, M)
    else:
        grad = z3.adjoint(idx, g[0], scale, M).unsqueeze(0)
    torch.cuda.synchronize()
    return zeta.cpu().numpy(), grad.cpu().numpy()


@pytest.mark.parametrize("nmaps,prec", [(1, "fp64"), (1, "mixed"), (5, "mixed")])
def test_autograd_forward_is_estimate_then_finalize(nmaps, prec):
    G.say("case: Zeta3Fn forward vs z3_estimate + z3_finalize", nmaps, prec)
    xyz, w, _ = pins.random_cap(2000, 4.0, 17)
    E = pins.small_edges(4, lo=0.1, hi=1.5, log=True)
    M = 5
    x = _maps(xyz, nmaps, 300)
    xs = x[0] if nmaps == 1 else x
    idx = G.build(xyz, xs.numpy(), E, w=w)
    zf = z3.Zeta3Fn.apply(xs.cuda(), idx, M, prec)
    ze, _ = _finalized(idx, M, prec)
    torch.cuda.synchronize()
    zf = zf.cpu().numpy().reshape(ze.shape)
    assert np.array_equal(zf, ze.cpu().numpy())
    assert np.abs(zf).max() > 0
    idx.free()


@pytest.mark.parametrize("nmaps,prec,shape", [(6, "mixed", (2, 16)), (6, "fp64", (2, 16)), (6, "mixed", None),
                                              (3, "mixed", None), (1, "mixed", None)])
def test_graph_replays_match_eager(nmaps, prec, shape):
    # six maps: the MFMA kernel (fixed block shape) or the register-tiled kernel in two groups
    G.say("case: graph step", nmaps, prec, shape)
    xyz, w, _ = pins.random_cap(3000, 5.0, 31)
    E = pins.small_edges(5, lo=0.1, hi=2.0, log=True)
    M = 6
    x0 = _maps(xyz, nmaps, 100)
    idx = G.build(xyz, x0.numpy(), E, w=w)
    ref_idx = G.build(xyz, x0.numpy(), E, w=w)
    if shape:
        idx.set_batch_shape(*shape)
        ref_idx.set_batch_shape(*shape)
    t = torch.from_numpy(np.random.default_rng(5).normal(size=(nmaps, M + 1, 5, 5, 2))).cuda() * 1e-3
    step = z3.GraphStep(idx, M, t, prec=prec)
    for r in range(3):
        x = _maps(xyz, nmaps, 200 + 10 * r)
        zeta_g, grad_g = step.run(x.cuda())
        torch.cuda.synchronize()
        zg, gg = zeta_g.cpu().numpy(), grad_g.cpu().numpy()
        ze, ge = _eager(ref_idx, x, M, prec, t)  # eager work between the replays
        G.say("replay", r, "zeta max", np.abs(ze).max(), "grad max", np.abs(ge).max())
        assert np.array_equal(zg, ze), r
        # the adjoint's FP64 atomics make its last bits depend on scheduling
        assert np.abs(gg - ge).max() <= 1e-12 * np.abs(ge).max(), r
    idx.free()
    ref_idx.free()
