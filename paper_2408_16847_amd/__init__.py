"""MI355X (gfx950) harmonic-basis 3PCF estimator: HIP kernels behind the libzeta3 C ABI."""

from ._lib import Zeta3Error  # noqa: F401
from .zeta3 import (GraphStep, Index, Zeta3Fn, accumulate, adjoint, adjoint_maps, contract, estimate,  # noqa: F401
                    estimate_cross, estimate_cross_catalogues, estimate_cross_raw,
                    estimate_maps, estimate_maps_raw, estimate_pivots, estimate_pivots_raw, estimate_raw,
                    profile_enable, profile_read, resum, sync)
