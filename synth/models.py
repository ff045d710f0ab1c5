"""Synthetic inputs of the FFTLog modelling workload (the line-of-sight integrals of the
modelling appendix): a linear power spectrum sampled on the appendix's log-spaced k grid,
a batch of line-of-sight kernels F(chi) = q_A q_B q_C D_+^4 on a log-spaced chi grid, and
an angle grid.

No cosmology is available here, so the stand-ins are analytic shapes with closed-form
transforms: P(k) = exp(-beta k^2) and F_b(chi) = chi^{p_b} exp(-chi / lam_b), with the
per-model (p_b, lam_b) drawn from a seeded generator.  This module draws and samples;
none of the FFTLog arithmetic (coefficients, Gamma factors, matrices) is here.
"""

from __future__ import annotations

import numpy as np


def log_grid(lo: float, hi: float, n: int) -> np.ndarray:
    """n log-spaced points from lo to hi, both ends included."""
    return lo * (hi / lo) ** (np.arange(n, dtype=np.float64) / (n - 1))


def fftlog_inputs(N: int = 256, k_min: float = 1e-6, k_max: float = 100.0, nchi: int = 512,
                  chi_min: float = 1e-4, chi_max: float = 60.0, nmodels: int = 4, ntheta: int = 64,
                  theta_min: float = 0.002, theta_max: float = 0.2, beta: float = 1.0, seed: int = 0):
    """Pk [N], F [nmodels, nchi], theta [ntheta] (radians), all FP64, plus the model
    parameters (p [nmodels], lam [nmodels]).  Model 0 is always (p, lam) = (3, 1)."""
    rng = np.random.default_rng(seed)
    k = log_grid(k_min, k_max, N)
    Pk = np.exp(-beta * k * k)
    p = rng.uniform(2.5, 4.0, nmodels)
    lam = rng.uniform(0.5, 2.0, nmodels)
    if nmodels:
        p[0], lam[0] = 3.0, 1.0
    chi = log_grid(chi_min, chi_max, nchi)
    F = chi[None, :] ** p[:, None] * np.exp(-chi[None, :] / lam[:, None])
    theta = log_grid(theta_min, theta_max, ntheta)
    return Pk, np.ascontiguousarray(F), theta, p, lam
