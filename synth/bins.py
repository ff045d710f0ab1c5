"""Radial bin edges.

The estimator bins neighbours by their angular distance from the pivot (the binned
multipoles of the estimator section; linear or logarithmic bins are both supported by
the paper's code).  Bin b is the half-open interval [theta_b, theta_{b+1}):

* linear: theta_b = theta_min + b (theta_max - theta_min) / nbins
* log:    theta_b = theta_min (theta_max / theta_min)^(b / nbins)

Every implementation receives the edges as a chord-squared table
E_b = (2 sin(theta_b / 2))^2, computed once here in FP64, so that all of them decide
bin membership against the very same numbers.
"""

from __future__ import annotations

import math

import numpy as np


def theta_edges(theta_min: float, theta_max: float, nbins: int, log: bool) -> np.ndarray:
    """Edges in radians, FP64, length nbins + 1."""
    if not (0.0 < theta_min < theta_max) or nbins < 1:
        raise ValueError("need 0 < theta_min < theta_max and nbins >= 1")
    b = np.arange(nbins + 1, dtype=np.float64)
    if log:
        e = theta_min * (theta_max / theta_min) ** (b / nbins)
    else:
        e = theta_min + b * (theta_max - theta_min) / nbins
    e[0], e[-1] = theta_min, theta_max
    return e


def chord2_edges(theta: np.ndarray) -> np.ndarray:
    """Chord-squared of angular edges: (2 sin(theta/2))^2, FP64."""
    s = 2.0 * np.sin(np.asarray(theta, dtype=np.float64) / 2.0)
    return s * s


def arcmin(x: float) -> float:
    return math.radians(x / 60.0)


def phi_boundaries(n_phi: int) -> np.ndarray:
    """Boundary directions of n_phi equal angular bins around a pivot: row k is
    (cos(2 pi k / n_phi), sin(2 pi k / n_phi)) in FP64 ([n_phi, 2]).

    Angular bin k holds the bearings [2 pi k / n_phi, 2 pi (k + 1) / n_phi), bearings
    measured from local north towards east.  Every implementation receives this table
    and decides bin membership by sign tests against these very numbers, as the radial
    bins are decided against the chord-squared table.
    """
    if n_phi < 4:
        raise ValueError("need n_phi >= 4")
    k = np.arange(n_phi, dtype=np.float64)
    t = 2.0 * np.pi * k / n_phi
    return np.ascontiguousarray(np.stack([np.cos(t), np.sin(t)], axis=1))
