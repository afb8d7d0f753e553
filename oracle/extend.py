"""FP64 oracle of the ConstrainedExtend step (test infrastructure only; see the package header).

Follows Alg. 2 ConstrainedExtend of arXiv 2604.13323 step by step, one extension at a time, with
the projections and collision checks of the oracle library (`Problem.project`, `Problem.check`).
The text of Sec. IV-A and IV-B fixes the steps; the points it leaves open are read as follows
(the same readings the library implements):

* the particles are spread along the extension direction only: p_i = q_steer + eps_i v, with the
  N(0, sigma^2) draws eps supplied by the caller;
* "succeeds the earliest" = the converged particle that needed the fewest Newton steps, the lowest
  index among equals;
* the n interpolated points of the second stage are the interior points k / (n + 1), k = 1..n,
  of the chord from q_start to q_proj;
* the recursive refinement inserts the projected midpoint of every gap of the chain, level after
  level, until no gap exceeds the resolution delta; at level l each gap next to a new point must be
  at most r / (n 2^l) (the second early exit's bound r / n, halved with every level);
* within one stage a non-converged point is reported before a collision, a collision before a
  gap; at the first stage a collision of q_proj is reported before the distance test.

Result codes: OK, ZERO (target equals start), NO_PARTICLE, COLLISION (of q_proj), TOO_FAR
(||q_proj - q_start|| > 2 dist), INTERP_FAILED, INTERP_COLLISION, GAP, numbered 0..7.
"""
from __future__ import annotations

import numpy as np

from . import CONVERGED

OK, ZERO, NO_PARTICLE, COLLISION, TOO_FAR, INTERP_FAILED, INTERP_COLLISION, GAP = range(8)


def extend_one(P, q_start, q_target, eps, r, delta, tol, max_iter, max_step=0.0, mode="stacked"):
    """One extension. Returns (code, particle index or -1, q_proj or None, chain [K, d] or None)."""
    s = np.asarray(q_start, np.float64)
    t = np.asarray(q_target, np.float64)
    eps = np.asarray(eps, np.float64)
    n = eps.size
    L = float(np.linalg.norm(t - s))
    if L == 0.0:
        return ZERO, -1, None, None
    # steer: a point at min(L, r) along the direction to the target
    dist = min(L, r)
    v = (t - s) / L
    q_steer = s + dist * v
    # first stage: n particles around q_steer along v, projected; keep the earliest success
    particles = q_steer[None, :] + eps[:, None] * v[None, :]
    qp, st, it, _ = P.project(particles, tol=tol, max_iter=max_iter, max_step=max_step, mode=mode)
    ok = np.flatnonzero(st == CONVERGED)
    if ok.size == 0:
        return NO_PARTICLE, -1, None, None
    best = int(ok[np.argmin(it[ok])])  # argmin returns the first (lowest index) among equal counts
    q_proj = qp[best]
    # first early exit: q_proj in collision, or projected too far from the start
    hit, _ = P.check(q_proj[None, :])
    if hit[0] != 0:
        return COLLISION, best, q_proj, None
    if np.linalg.norm(q_proj - s) > 2.0 * dist:
        return TOO_FAR, best, q_proj, None
    # second stage: interior points of the chord s -> q_proj, projected (level 0), then the
    # midpoints of every gap (levels 1, 2, ...) until the chain meets the resolution
    chain = [s, q_proj]
    level = 0
    while True:
        if level == 0:
            k = np.arange(1, n + 1) / (n + 1)
            new = s[None, :] + k[:, None] * (q_proj - s)[None, :]
        else:
            c = np.asarray(chain)
            new = 0.5 * (c[:-1] + c[1:])
        pn, stn, _, _ = P.project(new, tol=tol, max_iter=max_iter, max_step=max_step, mode=mode)
        if np.any(stn != CONVERGED):
            return INTERP_FAILED, best, q_proj, None
        hit, _ = P.check(pn)
        if np.any(hit != 0):
            return INTERP_COLLISION, best, q_proj, None
        if level == 0:
            chain = [s] + list(pn) + [q_proj]
        else:
            merged = []
            for a, m in zip(chain[:-1], pn):
                merged += [a, m]
            chain = merged + [chain[-1]]
        c = np.asarray(chain)
        gaps = np.linalg.norm(c[1:] - c[:-1], axis=1)
        # every gap of the chain touches a point added at this level
        if np.any(gaps > r / (n * 2.0 ** level)):
            return GAP, best, q_proj, None
        if gaps.max() <= delta:
            return OK, best, q_proj, c
        level += 1


def extend(P, q_start, q_target, eps, r, delta, tol=1e-6, max_iter=50, max_step=0.0, mode="stacked"):
    """E extensions (q_start, q_target [E, d], eps [E, n]). Returns dict with code [E] int8, particle
    [E] int32, q [E, d] (q_proj where a particle was selected, NaN elsewhere) and n_points [E] int32
    (chain length for OK, else 0)."""
    qs = np.asarray(q_start, np.float64)
    qt = np.asarray(q_target, np.float64)
    ep = np.asarray(eps, np.float64)
    E, d = qs.shape
    code = np.zeros(E, np.int8)
    part = np.full(E, -1, np.int32)
    q = np.full((E, d), np.nan)
    npts = np.zeros(E, np.int32)
    for e in range(E):
        c, b, qp, chain = extend_one(P, qs[e], qt[e], ep[e], r, delta, tol, max_iter, max_step, mode)
        code[e] = c
        part[e] = b
        if qp is not None:
            q[e] = qp
        if chain is not None:
            npts[e] = chain.shape[0]
    return dict(code=code, particle=part, q=q, n_points=npts)
