"""Launch-shape autotuning of the fused projection (a thin wrapper of the library's autotuner).

The persistent kernel's launch shape has three knobs: wavefronts per workgroup (1, 2, 4: how many
waves share a workgroup's LDS tile and its slice of the work queue), resident workgroups per CU (0 =
the occupancy limit) and lanes per configuration. The best shape depends on the family (register and
LDS footprint), the precision mode and the batch. `mc_autotune_project` times every candidate on a
real batch with HIP events, checks that all candidates give bit-identical outputs (the launch shape
must not change results) and keeps the fastest in the problem, where `project_batch` with the
variant and shape left at auto picks it up. Where the batch's exact-check queue is long (most
configurations near the obstacles), a second stage times the lane groups of the exact check (1, 2,
4, 8 or 16 lanes per configuration) in that shape and keeps the fastest for the problem's later
calls; the chosen size is the shape's `check_lanes` (0 when the queue was short).
"""
from __future__ import annotations


def tune(G, q, reps: int = 5, **kw) -> dict:
    """Time the candidate shapes on batch q (project options in kw: tol, max_iter, cond, check, mode)
    and store the fastest in problem G. Returns dict(best=shape, table=[shape + ms])."""
    best, table = G.autotune(q, reps=reps, **kw)
    return dict(best=best, table=[dict(shape, ms=ms) for shape, ms in table])


def tuned(G, dtype=None, mode="stacked") -> dict:
    """The shape stored in G for (dtype, mode), or {} (the library's defaults apply)."""
    import torch
    return G.tuned_shape(dtype or torch.float32, mode) or {}
