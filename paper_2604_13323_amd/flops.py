"""Algorithmic FLOP counts of one Newton iteration and of the final residual evaluation.

These are the operations the method has to perform per configuration (FMA = 2 FLOP),
counted from the scene's structure: forward kinematics once per iteration, the residual,
the Jacobian columns once, the Gram matrix J J^T over structural nonzeros, the Cholesky
factorisation and two triangular solves over the nonzeros of the factor, J^T y and the
update; and, once per configuration, the broad phase of the collision check (each link's
bounding sphere moved to the world frame and tested against the box around the obstacles).
Recomputations an implementation makes (the library re-runs the kinematics in its Gram and
J^T y passes to save registers, and once more in FP32 for the broad phase at convergence) are
not counted; sine/cosine, square roots and reciprocals count as one FLOP each.
"""
from __future__ import annotations

import numpy as np

from . import scenes as S


def _ancestor(parents, j, l):
    k = l
    while k >= 0:
        if k == j:
            return True
        k = parents[k]
    return False


def _block_rows(b, m_total):
    if b.btype in (S.BLK_POSE, S.BLK_REL):
        return bin(b.mask & 0x3F).count("1")
    if b.btype in (S.BLK_AXIS, S.BLK_COM, S.BLK_HULL):
        return 2
    if b.btype in (S.BLK_SPHERE, S.BLK_DIST):
        return 1
    return m_total


def jacobian_pattern(sc: S.Scene) -> np.ndarray:
    """Structural nonzero pattern of J (m x d) for kinematic scenes."""
    parents = [j.parent for j in sc.joints]
    rows = []
    for b in sc.blocks:
        nr = _block_rows(b, sc.m)
        comps = [c for c in range(6) if (b.mask >> c) & 1] if b.btype in (S.BLK_POSE, S.BLK_REL) else list(range(nr))
        for c in comps:
            row = np.zeros(sc.d, bool)
            for j in range(sc.d):
                jt = sc.joints[j].jtype
                if b.btype == S.BLK_POSE:
                    dep = _ancestor(parents, j, sc.frames[b.fa].link)
                elif b.btype in (S.BLK_REL, S.BLK_DIST):
                    dep = _ancestor(parents, j, sc.frames[b.fa].link) != _ancestor(parents, j, sc.frames[b.fb].link)
                elif b.btype == S.BLK_AXIS:
                    dep = _ancestor(parents, j, sc.frames[b.fa].link) and jt == S.JOINT_REV
                else:  # COM
                    dep = True
                if b.btype in (S.BLK_POSE, S.BLK_REL) and c >= 3 and jt == S.JOINT_PRI:
                    dep = False
                row[j] = dep
            rows.append(row)
    return np.array(rows)


def _chol_counts(Gnz: np.ndarray):
    m = Gnz.shape[0]
    L = np.tril(Gnz).copy()
    for k in range(m):
        for i in range(k + 1, m):
            for j in range(k + 1, i + 1):
                if L[i, k] and L[j, k]:
                    L[i, j] = True
    chol = 0
    for k in range(m):
        chol += 2  # square root and reciprocal
        below = [i for i in range(k + 1, m) if L[i, k]]
        chol += len(below)
        for i in below:
            chol += 2 * sum(1 for j in range(k + 1, i + 1) if L[j, k])
    offdiag = int(np.tril(L, -1).sum())
    solves = 2 * (2 * offdiag + m)
    return chol, solves


def iteration_flops(sc: S.Scene) -> dict:
    """Per-iteration FLOP components and the final-evaluation FLOPs for one configuration."""
    d, m = sc.d, sc.m
    if sc.family == S.FAMILY_SPHERE:
        res = 6
        it = dict(fk=0, residual=res, jacobian=3, gram=6, cholesky=2, solve=2, jty=6, update=4 * d)
        return dict(per_iter=sum(it.values()), final=res, parts=it)
    if sc.family == S.FAMILY_LINEAR:
        res = 2 * m * d + 2 * m
        gram = m * (m + 1) * d
        chol, solves = _chol_counts(np.ones((m, m), bool))
        it = dict(fk=0, residual=res, jacobian=0, gram=gram, cholesky=chol, solve=solves, jty=2 * m * d, update=4 * d)
        return dict(per_iter=sum(it.values()), final=res, parts=it)

    fk = 0
    for j, J in enumerate(sc.joints):
        rot = not np.allclose(J.R, np.eye(3))
        if J.parent >= 0:
            fk += 18 + (45 if rot else 0)
        fk += 18 if J.jtype == S.JOINT_REV else 6
        fk += 1 if J.jtype == S.JOINT_REV else 0  # sine and cosine
    frames = sum(18 + (0 if np.allclose(f.R, np.eye(3)) else 45) for f in sc.frames)
    massive = int(np.count_nonzero(sc.masses)) if sc.masses is not None else 0
    res = 0
    cols = 0
    Jp = jacobian_pattern(sc)
    for b in sc.blocks:
        if b.btype == S.BLK_POSE:
            res += 3 + 15 + 45 + 25
            cols += 45 + 20  # A = J_l^-1 W and J_l^-1
        elif b.btype == S.BLK_REL:
            res += 45 + 3 + 15 + 3 + 45 + 25
            cols += 45 + 20
        elif b.btype == S.BLK_COM:
            res += 24 * massive + 4
            cols += 6 * massive
        elif b.btype == S.BLK_HULL:  # CoM sums, then per polygon edge: side test, clamp, distance
            res += 24 * massive + 4 + 20 * b.aux
            cols += 6 * massive
        elif b.btype == S.BLK_DIST:  # difference, length, reciprocal, unit vector
            res += 3 + 5 + 1 + 3
    res += 2 * m  # norm
    r = 0
    for b in sc.blocks:
        nr = _block_rows(b, m)
        for j in range(d):
            dep = Jp[r:r + nr, j].any()
            if not dep:
                continue
            rev = sc.joints[j].jtype == S.JOINT_REV
            if b.btype in (S.BLK_POSE, S.BLK_REL):
                cols += 42 if rev else 15
            elif b.btype == S.BLK_AXIS:
                cols += 6
            elif b.btype == S.BLK_COM:
                cols += 17 if rev else 3
            elif b.btype == S.BLK_HULL:  # the CoM column and its 2 x 2 row map
                cols += (17 if rev else 3) + 6
            elif b.btype == S.BLK_DIST:  # u . (z x r) or u . z
                cols += 20 if rev else 5
        r += nr
    nnz_col = Jp.sum(axis=0)
    gram = int(sum(2 * k * (k + 1) // 2 for k in nnz_col))
    Gnz = (Jp.astype(int) @ Jp.T.astype(int)) > 0
    chol, solves = _chol_counts(Gnz)
    jty = 2 * int(Jp.sum())
    it = dict(fk=fk + frames, residual=res, jacobian=cols, gram=gram, cholesky=chol, solve=solves, jty=jty,
              update=4 * d)
    n_geo_links = len(set(int(l) for l in sc.spheres[:, 0] if l >= 0)) if sc.spheres is not None and len(sc.spheres) else 0
    broad = 35 * n_geo_links  # R c + p (18) and the box distance test (17) per link with spheres
    return dict(per_iter=sum(it.values()), final=fk + frames + res + broad, parts=dict(it, broad_once=broad))


def batch_flops(sc: S.Scene, iters: np.ndarray, with_broad: bool = True) -> float:
    """Algorithmic FLOPs of projecting a batch whose per-configuration step counts are `iters`
    (with_broad: including the collision broad phase of each configuration)."""
    f = iteration_flops(sc)
    iters = np.asarray(iters, np.int64)
    final = f["final"] - (0 if with_broad else f["parts"].get("broad_once", 0))
    return float(f["per_iter"] * iters.sum() + final * iters.size)


# Nominal per-unit figures: algorithmic FLOPs of one Newton iteration (structural sparsity
# counted, FMA = 2), by family.
NOMINAL_PER_ITER = {S.FAMILY_SPHERE: 15, S.FAMILY_ARM7_AXIS: 800, S.FAMILY_DUAL14_REL: 3300,
                   S.FAMILY_HUMANOID36: 13000}


def nominal_final_residual(sc: S.Scene) -> int:
    """One residual evaluation with the same per-unit figures: forward kinematics at ~96 FLOP per
    joint plus a sine/cosine per revolute joint, ~150 per pose or relative-pose block."""
    if not sc.joints:
        return iteration_flops(sc)["final"]
    n_rev = sum(1 for j in sc.joints if j.jtype == S.JOINT_REV)
    n_pose = sum(1 for b in sc.blocks if b.btype in (S.BLK_POSE, S.BLK_REL))
    return 96 * len(sc.joints) + n_rev + 150 * n_pose


def nominal_batch_flops(sc: S.Scene, iters: np.ndarray, with_broad: bool = True) -> float:
    """Algorithmic FLOPs of a batch with the nominal per-unit figures: per-iteration FLOPs x the
    batch's Newton iterations + one final residual per configuration (+ the broad phase of the
    collision check, from iteration_flops, when the launch runs it)."""
    iters = np.asarray(iters, np.int64)
    per_iter = NOMINAL_PER_ITER.get(sc.family, iteration_flops(sc)["per_iter"])
    broad = iteration_flops(sc)["parts"].get("broad_once", 0) if with_broad else 0
    return float(per_iter * iters.sum() + (nominal_final_residual(sc) + broad) * iters.size)
