"""paper_2406_16302_amd: the residual path estimator of "Residual path
integrals for re-rendering" (EGSR 2024) as a HIP library for one MI355X.

Python side = argument marshalling over the C ABI of librpi.so (include/rpi.h).
Every step of the estimator runs in the library's HIP kernels; there is no CPU
fallback.  PyTorch supplies device memory and streams.
"""
from .native import (FLAG_ACCUMULATE, FLAG_COUNT_WORK, FLAG_RECORDS, FLAG_TWO_WAY, RpiError, Scene, Edit,
                     Params, Proposal, autotune, load_library, render_frame, render_residual, render_residual_batch)

__all__ = ["Scene", "Edit", "Params", "Proposal", "render_residual", "render_frame", "render_residual_batch",
           "RpiError", "load_library", "autotune", "FLAG_TWO_WAY", "FLAG_ACCUMULATE", "FLAG_COUNT_WORK",
           "FLAG_RECORDS"]
