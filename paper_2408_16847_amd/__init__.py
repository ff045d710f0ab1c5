"""MI355X (gfx950) harmonic-basis 3PCF estimator: HIP kernels behind the libzeta3 C ABI."""

from .zeta3 import (Index, Zeta3Fn, accumulate, adjoint, contract, estimate, estimate_maps, estimate_maps_raw,  # noqa: F401
                    estimate_pivots, estimate_pivots_raw, estimate_raw, profile_enable, profile_read, resum,
                    sync)
