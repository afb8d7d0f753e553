"""Shared helpers of the GPU parity tests: build inputs with the oracle, run both sides, and
compare with the band rules.

Band rule (configurations excluded from exact status/iteration comparison, counted):
a configuration is in the band when the oracle's outcome changes if the tolerance moves by
+-0.1% (its residual sequence crosses tol within 0.1%: the GPU's FP64 residual differs from
the oracle's by ~1e-12 relative, so such a crossing can go either way), or when the oracle
needs at least max_iter - 1 steps.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2604_13323_amd import scenes as S

CONV, MAXIT, SING, DIV, NONF = range(5)


def config_inputs(name: str, small: bool = True, max_geo: int | None = None):
    """(scene, q_in [N, d] float64, geo_offsets, tol, max_iter): C2-C4 endpoints are projected by
    the oracle (FP64, tol 1e-10) and interpolated; C0/C1 come straight from the generator."""
    cfg = S.make_config(name, small=small)
    sc = cfg["scene"]
    P = oracle.Problem(sc.to_blob())
    offs = np.asarray(cfg["geo_offsets"], np.int32)
    if max_geo is not None and max_geo < len(offs) - 1:
        offs = offs[:max_geo + 1]
    if "q" in cfg:
        q = cfg["q"][:offs[-1]]
    else:
        e = cfg["endpoints"][:len(offs) - 1].reshape(-1, sc.d)
        qe = P.project(e, tol=1e-10, max_iter=100)[0]
        q = oracle.interpolate_interior(qe.reshape(-1, 2, sc.d), offs)
    return sc, P, q, offs, cfg["tol"], cfg["max_iter"]


def band_mask(P, q, tol, max_iter, max_step=0.0, mode="stacked", alpha=1.0, lam=0.0):
    """Configurations whose oracle outcome is not a well-posed target for exact comparison:
    the residual sequence crosses tol within +-0.1%; at least max_iter - 1 steps; an
    ill-conditioned path (sigma_min(J) < 1e-3 at some step, or a step longer than 1, where the
    linear model is far off and rounding differences send the iteration elsewhere on the
    manifold); or (with the divergence exit) a step within 1% of max_step."""
    lo = P.project(q, tol=tol * 0.999, max_iter=max_iter, max_step=max_step, mode=mode, alpha=alpha, lam=lam)
    hi = P.project(q, tol=tol * 1.001, max_iter=max_iter, max_step=max_step, path_info=True, mode=mode,
                   alpha=alpha, lam=lam)
    pi = hi[4]
    band = (lo[1] != hi[1]) | (lo[2] != hi[2]) | (hi[2] >= max_iter - 1)
    band |= pi[:, 0] < 1e-3
    if max_step > 0:
        # the path ends at the first long step: only a step within 1% of the threshold is ambiguous
        band |= np.abs(pi[:, 1] / max_step - 1.0) < 0.01
    else:
        band |= pi[:, 1] > 1.0
    return band


def to_dev(q: np.ndarray, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(q.T)).to(device="cuda", dtype=dtype)


def from_dev(t):
    return t.detach().cpu().numpy().astype(np.float64)
