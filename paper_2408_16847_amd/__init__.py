"""MI355X (gfx950) harmonic-basis 3PCF estimator: HIP kernels behind the libzeta3 C ABI."""

from .zeta3 import (Index, accumulate, contract, estimate, estimate_raw, profile_enable,  # noqa: F401
                    profile_read, resum, sync)
