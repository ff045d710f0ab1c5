"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package generates *inputs only*: HEALPix RING pixel centres, points on a
spherical cap, jittered grids on a plane, lognormal fields, radial-bin edge tables,
angular-bin boundary tables and the spectra and kernels of the FFTLog modelling workload.  It contains none of
the estimator's arithmetic (no pair search, no bearing, no multipoles, no
contraction), so both the CPU oracle and the GPU library can consume its arrays
without sharing any part of the method.
"""

from .healpix import npix, ring_centres, degrade_ring  # noqa: F401
from .fields import cap_points, plane_points, lognormal_field, field_params  # noqa: F401
from .bins import theta_edges, chord2_edges, phi_boundaries  # noqa: F401
from .models import log_grid, fftlog_inputs  # noqa: F401
from .configs import CONFIGS, Config, make_positions, make_values  # noqa: F401
