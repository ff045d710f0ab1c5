"""MI355X (gfx950) harmonic-basis 3PCF estimator: HIP kernels behind the libzeta3 C ABI."""

from ._lib import Zeta3Error  # noqa: F401
from .zeta3 import (GraphStep, Index, Zeta3Fn, accumulate, accumulate_hist, adjoint, adjoint_maps,  # noqa: F401
                    contract, estimate, estimate_hist, estimate_hist_raw, fftlog_a_functions, fftlog_workspace_size,
                    estimate_cross, estimate_cross_catalogues, estimate_cross_raw,
                    estimate_maps, estimate_maps_raw, estimate_pivots, estimate_pivots_raw, estimate_raw,
                    profile_enable, profile_read, resum, sync)
