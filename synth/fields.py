"""Seeded point catalogues and lognormal fields.

* ``cap_points``: points uniform on a spherical cap of radius ``radius_deg`` centred
  on (1, 0, 0).  cos(alpha) ~ U(cos radius, 1) and beta ~ U(0, 2 pi), drawn in that
  order from ``numpy.random.default_rng(1_000_000 + seed)``; the point is
  cos(alpha) x + sin(alpha) (cos(beta) y + sin(beta) z).
* ``lognormal_field``: delta(n) = exp(g(n) - var_g / 2) - 1 with
  g(n) = sum_k A_k cos(kappa_k n.u_k + psi_k).  The K mode parameters are drawn from
  ``numpy.random.default_rng(seed)`` in the order A ~ N(0, 0.3^2), kappa ~ U(lo, hi),
  u ~ normalised N(0, I_3), psi ~ U(0, 2 pi).  var_g is the ensemble variance given
  the draws, (1/2) sum_k A_k^2, so that <delta> = 0 over random phases.

These stand in for the weak-lensing convergence maps the paper measures (its
simulation section); the field is mean-zero and strongly skewed like a convergence map.
"""

from __future__ import annotations

import math

import numpy as np
import torch


def cap_points(n: int, radius_deg: float = 10.0, seed: int = 0, device="cpu") -> torch.Tensor:
    rng = np.random.default_rng(1_000_000 + seed)
    ca = rng.uniform(math.cos(math.radians(radius_deg)), 1.0, n)
    beta = rng.uniform(0.0, 2.0 * math.pi, n)
    sa = np.sqrt((1.0 - ca) * (1.0 + ca))
    xyz = np.stack([ca, sa * np.cos(beta), sa * np.sin(beta)])
    return torch.from_numpy(xyz).to(device)


def plane_points(side: int, jitter: float = 0.25, seed: int = 0, device="cpu") -> torch.Tensor:
    """side x side points on a plane, [2, n]: the unit grid (i, j) moved by a seeded uniform
    offset in [-jitter, jitter] per coordinate (a pixelised flat map), row-major in j then i."""
    rng = np.random.default_rng(3_000_000 + seed)
    i, j = np.meshgrid(np.arange(side, dtype=np.float64), np.arange(side, dtype=np.float64), indexing="xy")
    xy = np.stack([i.ravel(), j.ravel()])
    xy += rng.uniform(-jitter, jitter, size=xy.shape)
    return torch.from_numpy(xy).to(device)


def field_params(nmodes: int, kappa_lo: float, kappa_hi: float, seed: int):
    rng = np.random.default_rng(seed)
    amp = rng.normal(0.0, 0.3, nmodes)
    kappa = rng.uniform(kappa_lo, kappa_hi, nmodes)
    u = rng.normal(size=(nmodes, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    psi = rng.uniform(0.0, 2.0 * math.pi, nmodes)
    var_g = 0.5 * float(np.sum(amp * amp))
    return amp, kappa, u, psi, var_g


def gaussian_field(xyz: torch.Tensor, nmodes: int, kappa_lo: float, kappa_hi: float, seed: int,
                   chunk: int = 1 << 20) -> torch.Tensor:
    """g(n) = sum_k A_k cos(kappa_k n.u_k + psi_k) at the positions xyz [3, N] (FP64)."""
    amp, kappa, u, psi, _ = field_params(nmodes, kappa_lo, kappa_hi, seed)
    dev = xyz.device
    amp_t = torch.from_numpy(amp).to(dev)
    kap_t = torch.from_numpy(kappa).to(dev)
    u_t = torch.from_numpy(u).to(dev)
    psi_t = torch.from_numpy(psi).to(dev)
    n = xyz.shape[1]
    out = torch.empty(n, dtype=torch.float64, device=dev)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        proj = xyz[:, s:e].T @ u_t.T  # [chunk, K]
        out[s:e] = torch.cos(proj * kap_t + psi_t) @ amp_t
    return out


def lognormal_field(xyz: torch.Tensor, nmodes: int, kappa_lo: float, kappa_hi: float, seed: int,
                    fp32_values: bool = False) -> torch.Tensor:
    """delta = exp(g - var_g/2) - 1 (FP64); optionally rounded once to FP32 and promoted back."""
    *_, var_g = field_params(nmodes, kappa_lo, kappa_hi, seed)
    g = gaussian_field(xyz, nmodes, kappa_lo, kappa_hi, seed)
    delta = torch.expm1(g - 0.5 * var_g)
    if fp32_values:
        delta = delta.to(torch.float32).to(torch.float64)
    return delta
