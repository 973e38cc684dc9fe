"""MI355X (gfx950) library for the exact leave-one-out cross-validated
log-likelihood of the double-kernel conditional density estimator (Holmes,
Gray & Isbell, "Fast Nonparametric Conditional Density Estimation"), its
bandwidth gradient, and conditional density queries.

The computation runs in the HIP library ``libcde.so`` behind the C ABI of
``include/cde.h``; this package marshals arguments and hosts the drivers.
"""
from ._binding import CdeError, load  # noqa: F401
from .drivers import LooLogLik, ascend, normal_reference_bandwidths, select_grid  # noqa: F401
from .model import Model, argmax_first_finite, density_summary, launch_batch  # noqa: F401

__all__ = ["Model", "LooLogLik", "select_grid", "ascend", "normal_reference_bandwidths", "density_summary",
           "argmax_first_finite", "launch_batch", "CdeError", "load"]
