"""Seeded synthetic inputs (FV Laplacian systems in LDU form) shared by the
HIP path's tests and benchmark and by the CPU oracle's tests.

Pure NumPy/SciPy; holds none of the solver's arithmetic.
"""
from .configs import (Batch, Case, Piso, Transient, batch, cavity, concat, graded_spacing, laplace, make,  # noqa: F401
                      momentum, momentum_rhs, piso, transient, varcoef)
from . import mesh, rng  # noqa: F401
