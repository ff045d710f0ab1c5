"""The five synthetic workloads (sizes, binning, field recipe).

| name        | catalogue                           | field modes, kappa  | bins                 | m    |
|-------------|-------------------------------------|---------------------|----------------------|------|
| cap20k      | 20,000 points, 10 deg cap           | 64, U(20, 200)      | 10 linear 0.1-2 deg  | 0..8 |
| nside512    | HEALPix RING Nside 512 (3,145,728)  | 256, U(20, 800)     | 15 log 6'-300'       | 0..10|
| nside2048   | HEALPix RING Nside 2048 (50,331,648)| 512, U(50, 3000)    | 20 log 5'-200'       | 0..10|
| nside4096   | HEALPix RING Nside 4096 (201,326,592)| 1024, U(50, 3000)  | 20 log 2'-120'       | 0..10|
| batch64     | 64 maps at Nside 512, seeds 0..63   | as nside512         | as nside512          | 0..10|
| plane3m     | 1774 x 1774 jittered unit grid      | 256, U(0.04, 1.6)   | 15 log 1-40 units    | 0..10|

plane3m is the flat counterpart of nside512 (about the same number of points, spacing and
bins measured in spacings); its field is evaluated at (x, y, 0).

Weights are 1 and the field values are the x_i of the discrete field; for the two
largest maps the values are rounded once to FP32 (and promoted back to FP64), and
every implementation consumes those rounded values.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from .bins import arcmin, chord2_edges, theta_edges
from .fields import cap_points, lognormal_field, plane_points
from .healpix import ring_centres


@dataclass(frozen=True)
class Config:
    name: str
    kind: str            # "cap", "healpix" or "plane"
    n_or_nside: int
    nmodes: int
    kappa: tuple
    theta_min: float     # radians
    theta_max: float     # radians
    nbins: int
    log_bins: bool
    m_max: int
    fp32_values: bool = False
    nmaps: int = 1

    @property
    def npoints(self) -> int:
        if self.kind == "plane":
            return self.n_or_nside ** 2
        return self.n_or_nside if self.kind == "cap" else 12 * self.n_or_nside ** 2

    def theta_edges(self):
        return theta_edges(self.theta_min, self.theta_max, self.nbins, self.log_bins)

    def edges_chord2(self):
        """Edges of the pair test: chord squared on the sphere, distance squared on the plane."""
        if self.kind == "plane":
            return self.theta_edges() ** 2
        return chord2_edges(self.theta_edges())


CONFIGS = {
    "cap20k": Config("cap20k", "cap", 20_000, 64, (20.0, 200.0),
                     math.radians(0.1), math.radians(2.0), 10, False, 8),
    "nside512": Config("nside512", "healpix", 512, 256, (20.0, 800.0),
                       arcmin(6.0), arcmin(300.0), 15, True, 10),
    "nside2048": Config("nside2048", "healpix", 2048, 512, (50.0, 3000.0),
                        arcmin(5.0), arcmin(200.0), 20, True, 10, fp32_values=True),
    "nside4096": Config("nside4096", "healpix", 4096, 1024, (50.0, 3000.0),
                        arcmin(2.0), arcmin(120.0), 20, True, 10, fp32_values=True),
    "batch64": Config("batch64", "healpix", 512, 256, (20.0, 800.0),
                      arcmin(6.0), arcmin(300.0), 15, True, 10, nmaps=64),
    "plane3m": Config("plane3m", "plane", 1774, 256, (0.04, 1.6), 1.0, 40.0, 15, True, 10),
}


def make_positions(cfg: Config, device="cpu") -> torch.Tensor:
    if cfg.kind == "plane":
        return plane_points(cfg.n_or_nside, seed=0, device=device)
    if cfg.kind == "cap":
        return cap_points(cfg.n_or_nside, 10.0, seed=0, device=device)
    return ring_centres(cfg.n_or_nside, device=device)


def make_values(cfg: Config, xyz: torch.Tensor, seed: int = 0) -> torch.Tensor:
    if xyz.shape[0] == 2:  # plane: the field at (x, y, 0)
        xyz = torch.cat([xyz, torch.zeros_like(xyz[:1])])
    return lognormal_field(xyz, cfg.nmodes, cfg.kappa[0], cfg.kappa[1], seed,
                           fp32_values=cfg.fp32_values)
