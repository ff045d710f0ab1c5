"""HEALPix RING-scheme pixel centres, written from the published pixelisation formulas.

The paper analyses full-sky HEALPix maps (Introduction and the simulation section:
Nside = 4096, 0.86 arcmin pixels, 201,326,592 pixels).  healpy is not available, so
the pixel centres are generated here from the equal-area ring geometry published by
Gorski et al. (2005, ApJ 622, 759):

* rings i = 1 .. 4 Nside - 1 ordered from the north pole;
* north polar cap (i < Nside): 4 i pixels, z = 1 - i^2 / (3 Nside^2),
  phi_j = (pi / 2i) (j - 1/2), j = 1 .. 4i;
* equatorial belt (Nside <= i <= 3 Nside): 4 Nside pixels, z = 4/3 - 2 i / (3 Nside),
  phi_j = (pi / 2 Nside) (j - s/2) with s = (i - Nside + 1) mod 2 (for s = 0 the
  ring is indexed from phi = 0, i.e. phi_j = (pi / 2 Nside)(j - 1), which is the same
  set of centres in the standard RING order);
* south polar cap: mirror image of the north cap (z -> -z).

RING pixel indices run ring by ring, and within a ring in increasing phi.
Everything is FP64.  The functions run on any torch device; a run generates its
inputs once and hands the same arrays to every implementation.
"""

from __future__ import annotations

import math

import torch


def npix(nside: int) -> int:
    return 12 * nside * nside


def _ring_table(nside: int, device):
    """Per-ring (start, count, z, 1-|z|, sin(theta), phase offset), FP64/int64."""
    n = nside
    i = torch.arange(1, 4 * n, dtype=torch.int64, device=device)  # ring numbers
    north = i < n
    south = i > 3 * n
    ip = torch.where(south, 4 * n - i, i)  # ring number counted from the nearer pole
    cap = north | south
    count = torch.where(cap, 4 * ip, torch.full_like(i, 4 * n))
    start = torch.cumsum(count, 0) - count
    ipd = ip.to(torch.float64)
    omz_cap = ipd * ipd / (3.0 * n * n)  # 1 - |z| exactly in the caps
    z_belt = 4.0 / 3.0 - 2.0 * i.to(torch.float64) / (3.0 * n)
    z = torch.where(north, 1.0 - omz_cap, torch.where(south, -(1.0 - omz_cap), z_belt))
    omz = torch.where(cap, omz_cap, 1.0 - z_belt.abs())
    # sin(theta) = sqrt((1 - z)(1 + z)); in the caps use 1 - |z| directly
    sin_cap = torch.sqrt(omz_cap * (2.0 - omz_cap))
    sin_belt = torch.sqrt((1.0 - z_belt) * (1.0 + z_belt))
    sint = torch.where(cap, sin_cap, sin_belt)
    # belt rings alternate between centres at phi = (j - 1/2) dphi and (j - 1) dphi; the
    # latter is the paper's (j - s/2) rule with s = 0, indexed from phi = 0 as in the
    # standard RING numbering
    s = torch.remainder(i - n + 1, 2).to(torch.float64)
    off = torch.where(cap, torch.full_like(z, 0.5), 1.0 - 0.5 * s)
    return start, count, z, omz, sint, off


def ring_centres(nside: int, device="cpu", with_ring=False):
    """FP64 unit vectors of all RING pixel centres, shape [3, 12 Nside^2].

    With ``with_ring=True`` also returns (ring index 0-based per pixel, z, 1-|z|, phi).
    """
    if nside < 1:
        raise ValueError("nside must be >= 1")
    start, count, z, omz, sint, off = _ring_table(nside, device)
    nr = count.numel()
    ring = torch.repeat_interleave(torch.arange(nr, device=device), count)
    j = torch.arange(npix(nside), dtype=torch.int64, device=device) - start[ring] + 1
    phi = (2.0 * math.pi / count[ring].to(torch.float64)) * (j.to(torch.float64) - off[ring])
    st = sint[ring]
    xyz = torch.empty((3, phi.numel()), dtype=torch.float64, device=device)
    xyz[0] = st * torch.cos(phi)
    xyz[1] = st * torch.sin(phi)
    xyz[2] = z[ring]
    if with_ring:
        return xyz, ring, z[ring], omz[ring], phi
    return xyz


def ang2pix_ring(nside: int, z: torch.Tensor, omz: torch.Tensor, phi: torch.Tensor) -> torch.Tensor:
    """RING pixel index containing (z, phi); ``omz`` = 1 - |z| given separately for accuracy.

    Restates the published HEALPix point-to-pixel rule: equatorial points are located
    by the two families of pixel-boundary lines z = 4/3 -/+ 8 phi' / (3 pi) ...,
    polar points by the lines through the pole in the (phi, sqrt(1-|z|)) plane.
    """
    n = nside
    tt = torch.remainder(phi, 2.0 * math.pi) / (0.5 * math.pi)  # in [0, 4)
    za = z.abs()
    # equatorial belt
    t1 = n * (0.5 + tt)
    t2 = n * z * 0.75
    jp = torch.floor(t1 - t2).to(torch.int64)
    jm = torch.floor(t1 + t2).to(torch.int64)
    ir = n + 1 + jp - jm
    kshift = 1 - (ir & 1)
    ipix = torch.div(jp + jm - n + kshift + 1, 2, rounding_mode="floor")
    ipix = torch.remainder(ipix, 4 * n)
    ncap = 2 * n * (n - 1)
    pix_eq = ncap + (ir - 1) * 4 * n + ipix
    # polar caps
    tp = tt - torch.floor(tt)
    tmp = n * torch.sqrt(3.0 * omz)
    jp2 = torch.floor(tp * tmp).to(torch.int64)
    jm2 = torch.floor((1.0 - tp) * tmp).to(torch.int64)
    ir2 = jp2 + jm2 + 1
    ip2 = torch.floor(tt * ir2.to(torch.float64)).to(torch.int64)
    ip2 = torch.remainder(ip2, 4 * ir2)
    pix_n = 2 * ir2 * (ir2 - 1) + ip2
    pix_s = npix(n) - 2 * ir2 * (ir2 + 1) + ip2
    pix_cap = torch.where(z > 0, pix_n, pix_s)
    return torch.where(za <= 2.0 / 3.0, pix_eq, pix_cap)


def degrade_ring(nside: int, values: torch.Tensor, weights: torch.Tensor | None = None):
    """Average an Nside RING map onto Nside/2 (the coarse neighbour catalogue).

    Returns (parent positions [3, Npix/4], parent values = mean of the 4 children,
    parent weights = sum of the children's weights).  The parent of each child is the
    Nside/2 pixel that contains the child's centre.
    """
    if nside % 2:
        raise ValueError("nside must be even to degrade")
    device = values.device
    _, _, z, omz, phi = ring_centres(nside, device=device, with_ring=True)
    parent = ang2pix_ring(nside // 2, z, omz, phi)
    del z, omz, phi
    npar = npix(nside // 2)
    w = torch.ones_like(values) if weights is None else weights
    # group the children of each parent in a fixed order (deterministic sums)
    order = torch.argsort(parent, stable=True)
    ps = parent[order].view(npar, 4)
    if not bool((ps == torch.arange(npar, device=device).unsqueeze(1)).all()):
        raise RuntimeError("degrade: a parent pixel did not receive exactly 4 children")
    vc = values[order].view(npar, 4)
    wc = w[order].view(npar, 4)
    vmean = (((vc[:, 0] + vc[:, 1]) + vc[:, 2]) + vc[:, 3]) / 4.0
    wsum = ((wc[:, 0] + wc[:, 1]) + wc[:, 2]) + wc[:, 3]
    return ring_centres(nside // 2, device=device), vmean, wsum
