"""Batched manifold projection for AMD MI355X (gfx950): HIP kernels behind a C ABI.

The method is the projection step of arXiv 2604.13323 (Alg. 2 ParallelProject with
min-norm Newton steps on the stacked constraint, followed by the sphere collision
check), plus a vector-Jacobian product through the converged projection.
"""
from .binding import (CONVERGED, COLLIDES, DIVERGED, FREE, MAX_ITER, NONFINITE, SINGULAR, UNCHECKED,  # noqa: F401
                      McError, PathLengthFn, Problem, ProjectFn, ProjectResult, lib, project)
