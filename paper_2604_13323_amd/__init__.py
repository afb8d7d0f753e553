"""Batched manifold projection for AMD MI355X (gfx950): HIP kernels behind a C ABI.

The method is the projection step of arXiv 2604.13323 (Alg. 2 ParallelProject with
min-norm Newton steps on the stacked constraint, followed by the sphere collision
check), a vector-Jacobian product through the converged projection, and the batched
ConstrainedExtend step of Alg. 2 built on the projection.
"""
from .binding import (CONVERGED, COLLIDES, DIVERGED, FREE, MAX_ITER, NONFINITE, SINGULAR, UNCHECKED,  # noqa: F401
                      EXT_COLLISION, EXT_GAP, EXT_INTERP_COLLISION, EXT_INTERP_FAILED, EXT_NO_PARTICLE, EXT_OK,
                      EXT_TOO_FAR, EXT_ZERO, ExtendResult, McError, PathLengthFn, Problem, ProjectFn, ProjectResult,
                      lib, project)
