"""Seeded synthetic scenes and raw workloads for the batched manifold projection.

This module only *writes inputs*: robot descriptions (joint tree, link masses,
collision spheres), constraint-block specifications, obstacle spheres, and raw
(unprojected) configurations. It holds none of the method's arithmetic: no
forward kinematics, no residuals, no Jacobians, no projection and no collision
test. Both the FP64 oracle and the HIP library read the same serialized scene
blob and implement the method independently.

Kinematic convention (shared *specification*, implemented separately by each
side): joint j has a parent joint p(j) (-1 = world), a fixed origin transform
O_j = (R_o, p_o) and an axis a_j in {x, y, z} of its own frame. The frame of
link j is T_j = T_p(j) * O_j * Q_j(q_j), where Q_j rotates about a_j by q_j
(revolute) or translates along a_j by q_j (prismatic). Joints are listed in
depth-first preorder, so every subtree is a contiguous index range.

The constraint blocks follow the paper: a TSR pose error (Eq. 1, with the TSR
frame T_w^0 = T_ref and the grasp offset folded into the end-effector frame),
optionally with finite bounds B^w per component (Sec. III), a relative pose
error between two end-effectors (Eq. 2), the centre-of-mass xy error of the
humanoid's stability constraint (the Digit constraint figure) in two forms,
equality to the support-polygon centroid and distance to the support polygon,
the closed-linkage rod lengths of the same figure, plus the synthetic sphere,
axis-alignment and linear constraints used for closed-form checks.

RNG: numpy PCG64 seeded with [config_id, stream]; streams 0 robot, 1 obstacles,
2 workload, 3 finite-difference sample, 4 geodesic lengths, 5 extension particle draws,
6 reference configuration of the bounded-TSR arm.
"""
from __future__ import annotations

import math
import struct
from dataclasses import dataclass, field

import numpy as np

# ---- enums (must match include/mcproj.h) ---------------------------------
FAMILY_SPHERE = 0
FAMILY_LINEAR = 1
FAMILY_PLANAR2 = 2
FAMILY_ARM7_AXIS = 3
FAMILY_DUAL14_REL = 4
FAMILY_HUMANOID36 = 5
FAMILY_DIGIT36 = 6
FAMILY_ARM7_TSR = 7
FAMILY_NAMES = {
    FAMILY_SPHERE: "sphere3",
    FAMILY_LINEAR: "linear",
    FAMILY_PLANAR2: "planar2",
    FAMILY_ARM7_AXIS: "arm7_axis",
    FAMILY_DUAL14_REL: "dual14_rel",
    FAMILY_HUMANOID36: "humanoid36",
    FAMILY_DIGIT36: "digit36",
    FAMILY_ARM7_TSR: "arm7_tsr",
}

JOINT_REV = 0
JOINT_PRI = 1

BLK_POSE = 0    # TSR pose error of one frame against a fixed target (Eq. 1)
BLK_REL = 1     # relative pose error of frame b seen from frame a (Eq. 2)
BLK_AXIS = 2    # frame z-axis parallel to world z: rows (z_x, z_y)
BLK_COM = 3     # centre-of-mass xy minus a target point
BLK_SPHERE = 4  # q.q - 1
BLK_LINEAR = 5  # A q - b
BLK_DIST = 6    # closed linkage: ||p_b - p_a|| - L between the origins of frames a and b (L in target[0])
BLK_HULL = 7    # centre-of-mass xy minus its nearest point of a convex polygon (zero inside)

POSE_BOUNDED = 1  # Block.aux flag of a POSE block: rows are the excess over [lo, hi] (ext[0:6], ext[6:12])
MAX_HULL_VERTICES = 8

MAGIC = 0x5343434D  # 'MCCS'
VERSION = 1          # version 2: every block record is followed by 16 doubles of block data (ext)
HEADER_INTS = 16
N_EXT = 16

# obstacle-free joint limits are not part of the method; none are stored.

CONFIG_IDS = {"c0": 0, "c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5, "c6": 6}


def rng_for(config_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(config_id), int(stream)])


@dataclass
class Joint:
    parent: int
    jtype: int
    axis: int
    R: np.ndarray  # 3x3 origin rotation
    p: np.ndarray  # origin translation


@dataclass
class Frame:
    link: int
    R: np.ndarray
    p: np.ndarray


@dataclass
class Block:
    btype: int
    fa: int = -1
    fb: int = -1
    mask: int = 0x3F
    ref_from_qref: int = 0
    R: np.ndarray = field(default_factory=lambda: np.eye(3))
    p: np.ndarray = field(default_factory=lambda: np.zeros(3))
    target: np.ndarray = field(default_factory=lambda: np.zeros(3))
    aux: int = 0        # POSE: POSE_BOUNDED; HULL: number of polygon vertices
    ext: np.ndarray = field(default_factory=lambda: np.zeros(N_EXT))  # POSE bounds lo[6], hi[6]; HULL xy vertices


@dataclass
class Scene:
    family: int
    d: int
    m: int
    joints: list = field(default_factory=list)
    masses: np.ndarray = None      # (n_joints,)
    coms: np.ndarray = None        # (n_joints, 3) link CoM in link frame
    frames: list = field(default_factory=list)
    blocks: list = field(default_factory=list)
    spheres: np.ndarray = None     # (S, 5): link, cx, cy, cz, r   (link -1: the configuration point itself)
    obstacles: np.ndarray = None   # (O, 4): x, y, z, r
    qref: np.ndarray = None        # (d,) reference configuration for blocks with ref_from_qref
    A: np.ndarray = None           # (m, d) for BLK_LINEAR
    b: np.ndarray = None           # (m,)
    name: str = ""

    def to_blob(self) -> bytes:
        nj = len(self.joints)
        S = 0 if self.spheres is None else len(self.spheres)
        O = 0 if self.obstacles is None else len(self.obstacles)
        has_qref = 1 if self.qref is not None else 0
        has_lin = 1 if self.A is not None else 0
        v2 = any(b.aux != 0 or np.any(np.asarray(b.ext) != 0) for b in self.blocks)
        hdr = [MAGIC, 2 if v2 else VERSION, self.family, self.d, self.m, nj, len(self.frames),
               len(self.blocks), S, O, has_qref, has_lin, 0, 0, 0, 0]
        out = [struct.pack("<16i", *hdr)]
        for j in self.joints:
            out.append(struct.pack("<4i", j.parent, j.jtype, j.axis, 0))
            out.append(np.asarray(j.R, "<f8").reshape(9).tobytes())
            out.append(np.asarray(j.p, "<f8").reshape(3).tobytes())
        for k in range(nj):
            out.append(struct.pack("<d", float(self.masses[k])))
            out.append(np.asarray(self.coms[k], "<f8").reshape(3).tobytes())
        for f in self.frames:
            out.append(struct.pack("<2i", f.link, 0))
            out.append(np.asarray(f.R, "<f8").reshape(9).tobytes())
            out.append(np.asarray(f.p, "<f8").reshape(3).tobytes())
        for b in self.blocks:
            out.append(struct.pack("<6i", b.btype, b.fa, b.fb, b.mask, b.ref_from_qref, b.aux))
            out.append(np.asarray(b.R, "<f8").reshape(9).tobytes())
            out.append(np.asarray(b.p, "<f8").reshape(3).tobytes())
            out.append(np.asarray(b.target, "<f8").reshape(3).tobytes())
            if v2:
                out.append(np.asarray(b.ext, "<f8").reshape(N_EXT).tobytes())
        for s in (self.spheres if S else []):
            out.append(struct.pack("<2i", int(s[0]), 0))
            out.append(np.asarray(s[1:5], "<f8").tobytes())
        for o in (self.obstacles if O else []):
            out.append(np.asarray(o, "<f8").reshape(4).tobytes())
        if has_qref:
            out.append(np.asarray(self.qref, "<f8").reshape(self.d).tobytes())
        if has_lin:
            out.append(np.asarray(self.A, "<f8").reshape(self.m * self.d).tobytes())
            out.append(np.asarray(self.b, "<f8").reshape(self.m).tobytes())
        return b"".join(out)


# ---- small rigid-transform constructors (closed forms, data only) --------
def rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)


def rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=np.float64)


def dh_origin(a, d, alpha):
    """Fixed part of a standard DH link, Tz(d) Tx(a) Rx(alpha): rotation Rx(alpha), translation (a, 0, d)."""
    return rot_x(alpha), np.array([a, 0.0, d])


def _uniform_sphere_points(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def bounded_pose_block(fa: int, lo, hi, R=None, p=None, mask: int = 0x3F) -> Block:
    """TSR pose block (Eq. 1) with finite bounds B^w: component c of [t; log(R)^v] is constrained to
    [lo[c], hi[c]] (+-inf for a free component)."""
    ext = np.zeros(N_EXT)
    ext[0:6] = np.asarray(lo, np.float64)
    ext[6:12] = np.asarray(hi, np.float64)
    return Block(BLK_POSE, fa=fa, mask=mask, R=np.eye(3) if R is None else np.asarray(R, np.float64),
                 p=np.zeros(3) if p is None else np.asarray(p, np.float64), aux=POSE_BOUNDED, ext=ext)


def hull_block(vertices) -> Block:
    """Centre-of-mass block against a convex polygon given counter-clockwise (3 to 8 xy vertices)."""
    v = np.asarray(vertices, np.float64).reshape(-1, 2)
    assert 3 <= len(v) <= MAX_HULL_VERTICES
    ext = np.zeros(N_EXT)
    ext[:2 * len(v)] = v.reshape(-1)
    return Block(BLK_HULL, aux=len(v), ext=ext)


def dist_block(fa: int, fb: int, length: float = 0.0, from_qref: bool = False) -> Block:
    """Closed-linkage block: the distance between the origins of frames fa and fb equals `length`, or
    the distance at q_ref when from_qref is set."""
    return Block(BLK_DIST, fa=fa, fb=fb, target=np.array([float(length), 0.0, 0.0]),
                 ref_from_qref=1 if from_qref else 0)


def convex_hull_ccw(points) -> np.ndarray:
    """Counter-clockwise convex hull of 2-D points (Andrew's monotone chain), collinear points dropped."""
    P = sorted({(float(x), float(y)) for x, y in np.asarray(points, np.float64).reshape(-1, 2)})

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for pt in P:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], pt) <= 0:
            lower.pop()
        lower.append(pt)
    for pt in reversed(P):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], pt) <= 0:
            upper.pop()
        upper.append(pt)
    return np.array(lower[:-1] + upper[:-1])


# ---- C0: toy sphere -------------------------------------------------------
def sphere_scene(config_id: int = 0, n_obstacles: int = 64) -> Scene:
    r = rng_for(config_id, 1)
    obs = np.empty((n_obstacles, 4))
    obs[:, :3] = r.uniform(-1.5, 1.5, (n_obstacles, 3))
    obs[:, 3] = r.uniform(0.05, 0.2, n_obstacles)
    return Scene(family=FAMILY_SPHERE, d=3, m=1, joints=[], masses=np.zeros(0), coms=np.zeros((0, 3)),
                 blocks=[Block(BLK_SPHERE)], spheres=np.array([[-1, 0, 0, 0, 0.0]]), obstacles=obs,
                 name="sphere3")


def sphere_workload(config_id: int = 0, n_seg: int = 1024, step: float = 0.05, noise: float = 0.05):
    """Chords between random unit-sphere points, sampled at spacing <= step, each point perturbed by N(0, noise^2).

    Returns (q [N,3] float64, geo_offsets [n_seg+1] int32)."""
    r = rng_for(config_id, 2)
    a = _uniform_sphere_points(r, n_seg)
    b = _uniform_sphere_points(r, n_seg)
    qs, offs = [], [0]
    for k in range(n_seg):
        L = float(np.linalg.norm(b[k] - a[k]))
        npts = int(math.ceil(L / step)) + 1
        t = np.arange(npts) / (npts - 1)
        qs.append(a[k][None, :] + t[:, None] * (b[k] - a[k])[None, :])
        offs.append(offs[-1] + npts)
    q = np.concatenate(qs, 0)
    q = q + r.normal(0.0, noise, q.shape)
    return q, np.asarray(offs, np.int32)


# ---- linear and planar test scenes (closed-form pins) --------------------
def linear_scene(A, b) -> Scene:
    A = np.asarray(A, np.float64)
    b = np.asarray(b, np.float64)
    m, d = A.shape
    return Scene(family=FAMILY_LINEAR, d=d, m=m, joints=[], masses=np.zeros(0), coms=np.zeros((0, 3)),
                 blocks=[Block(BLK_LINEAR)], spheres=np.zeros((0, 5)), obstacles=np.zeros((0, 4)),
                 A=A, b=b, name="linear")


def planar2_scene(l1: float, l2: float, target_xy) -> Scene:
    """Planar 2R arm about world z; constraint: tip position (x, y) equals the target (POSE block, mask x|y)."""
    I = np.eye(3)
    joints = [Joint(-1, JOINT_REV, 2, I, np.zeros(3)),
              Joint(0, JOINT_REV, 2, I, np.array([l1, 0.0, 0.0]))]
    frames = [Frame(1, I, np.array([l2, 0.0, 0.0]))]
    blk = Block(BLK_POSE, fa=0, mask=0x3, p=np.array([target_xy[0], target_xy[1], 0.0]))
    spheres = np.array([[0, l1 * t, 0, 0, 0.02] for t in (0.0, 0.5, 1.0)] +
                       [[1, l2 * t, 0, 0, 0.02] for t in (0.0, 0.5, 1.0)], np.float64)
    return Scene(family=FAMILY_PLANAR2, d=2, m=2, joints=joints, masses=np.ones(2), coms=np.zeros((2, 3)),
                 frames=frames, blocks=[blk], spheres=spheres, obstacles=np.zeros((0, 4)), name="planar2")


# ---- C1: 7-DoF DH arm, end-effector z parallel to world z ----------------
def _dh_params(r, n=7):
    a = r.uniform(0.1, 0.4, n)
    d = r.uniform(0.1, 0.4, n)
    alpha = r.choice([0.0, math.pi / 2, -math.pi / 2], n)
    # at least two twisted axes, so the arm is not planar (data recipe, not a method step)
    if np.count_nonzero(alpha[:n - 1]) < 2:
        alpha[1] = math.pi / 2
        alpha[3] = -math.pi / 2
    return a, d, alpha


def _dh_chain(a, d, alpha, base_p, parent0=-1, index0=0):
    """Joints for a standard-DH serial chain, converted to origin/axis form.

    Joint i rotates about its own z; its origin is the fixed part of the previous DH link.
    Returns (joints, link sphere segments, end-effector frame offset)."""
    joints = []
    n = len(a)
    for i in range(n):
        if i == 0:
            R, p = np.eye(3), np.asarray(base_p, np.float64)
            parent = parent0
        else:
            R, p = dh_origin(a[i - 1], d[i - 1], alpha[i - 1])
            parent = index0 + i - 1
        joints.append(Joint(parent, JOINT_REV, 2, R, p))
    segs = [np.array([a[i], 0.0, d[i]]) for i in range(n)]   # link i spans origin -> next origin
    ee_R, ee_p = dh_origin(a[n - 1], d[n - 1], alpha[n - 1])
    return joints, segs, (ee_R, ee_p)


def _link_spheres(link, seg, k, radius, start=None):
    start = np.zeros(3) if start is None else np.asarray(start, np.float64)
    ts = np.linspace(0.0, 1.0, k)
    return [[link, *(start + t * (np.asarray(seg) - start)), radius] for t in ts]


def arm7_axis_scene(config_id: int = 1, n_obstacles: int = 200) -> Scene:
    r = rng_for(config_id, 0)
    a, d, alpha = _dh_params(r)
    joints, segs, (eeR, eep) = _dh_chain(a, d, alpha, np.zeros(3))
    spheres = []
    for i in range(7):
        spheres += _link_spheres(i, segs[i], 4, 0.05)
    ro = rng_for(config_id, 1)
    Rw = 0.6 * float(np.sum(a + d))
    obs = np.empty((n_obstacles, 4))
    obs[:, :3] = ro.uniform(-Rw, Rw, (n_obstacles, 3))
    obs[:, 3] = ro.uniform(0.05, 0.2, n_obstacles)
    masses = r.uniform(0.5, 2.0, 7)
    coms = np.array([0.5 * s for s in segs])
    return Scene(family=FAMILY_ARM7_AXIS, d=7, m=2, joints=joints, masses=masses, coms=coms,
                 frames=[Frame(6, eeR, eep)], blocks=[Block(BLK_AXIS, fa=0)],
                 spheres=np.array(spheres, np.float64), obstacles=obs, name="arm7_axis")


# TSR of the arm-with-bounds batch (Sec. III, the upright-mug example): the TSR frame is the
# end-effector pose at a reference configuration, the bounds B^w let the frame translate by up to
# 0.1 m in x and y and 0.02 m in z and rotate by up to 0.05 rad about x and y (tilt) and 0.5 rad about z
ARM7_TSR_LO = np.array([-0.1, -0.1, -0.02, -0.05, -0.05, -0.5])
ARM7_TSR_HI = np.array([0.1, 0.1, 0.02, 0.05, 0.05, 0.5])


def arm7_tsr_scene(config_id: int = 6, n_obstacles: int = 200) -> Scene:
    """The 7-DoF DH arm of the C1 recipe (its own seed) with one TSR pose block with finite bounds on
    its end-effector frame; T_w^0 is the end-effector pose at q_ref ~ U[-pi, pi]^7 (stream 6)."""
    base = arm7_axis_scene(config_id, n_obstacles)
    blk = bounded_pose_block(0, ARM7_TSR_LO, ARM7_TSR_HI)
    blk.ref_from_qref = 1
    qref = rng_for(config_id, 6).uniform(-math.pi, math.pi, 7)
    return Scene(family=FAMILY_ARM7_TSR, d=7, m=6, joints=base.joints, masses=base.masses, coms=base.coms,
                 frames=base.frames, blocks=[blk], spheres=base.spheres, obstacles=base.obstacles, qref=qref,
                 name="arm7_tsr")


def arm7_workload(config_id: int = 1, n_seg: int = 4096, n_pts: int = 32, noise: float = 0.1):
    """Segments between joint vectors uniform in [-pi, pi]^7, n_pts points each (endpoints included),
    plus N(0, noise^2) joint noise per point. Returns (q [N,7], geo_offsets)."""
    r = rng_for(config_id, 2)
    a = r.uniform(-math.pi, math.pi, (n_seg, 7))
    b = r.uniform(-math.pi, math.pi, (n_seg, 7))
    t = np.arange(n_pts) / (n_pts - 1)
    q = a[:, None, :] + t[None, :, None] * (b - a)[:, None, :]
    q = q.reshape(-1, 7) + r.normal(0.0, noise, (n_seg * n_pts, 7))
    offs = np.arange(n_seg + 1, dtype=np.int32) * n_pts
    return q, offs


# ---- C2: dual 7-DoF arms, fixed relative end-effector pose ---------------
def dual14_rel_scene(config_id: int = 2, n_obstacles: int = 400) -> Scene:
    r = rng_for(config_id, 0)
    aL, dL, alL = _dh_params(r)
    aR, dR, alR = _dh_params(r)
    jL, segL, (eRL, epL) = _dh_chain(aL, dL, alL, np.array([0.0, 0.3, 0.0]), -1, 0)
    jR, segR, (eRR, epR) = _dh_chain(aR, dR, alR, np.array([0.0, -0.3, 0.0]), -1, 7)
    joints = jL + jR
    spheres = []
    for i in range(7):
        spheres += _link_spheres(i, segL[i], 4, 0.05)
    for i in range(7):
        spheres += _link_spheres(7 + i, segR[i], 4, 0.05)
    qref = r.uniform(-math.pi, math.pi, 14)
    ro = rng_for(config_id, 1)
    Rw = 0.6 * float(max(np.sum(aL + dL), np.sum(aR + dR)))
    obs = np.empty((n_obstacles, 4))
    obs[:, :3] = ro.uniform(-Rw, Rw, (n_obstacles, 3))
    obs[:, 3] = ro.uniform(0.05, 0.2, n_obstacles)
    masses = r.uniform(0.5, 2.0, 14)
    coms = np.array([0.5 * s for s in segL + segR])
    # the grasp: relative pose of the right end-effector seen from the left one at q_ref
    blk = Block(BLK_REL, fa=0, fb=1, ref_from_qref=1)
    return Scene(family=FAMILY_DUAL14_REL, d=14, m=6, joints=joints, masses=masses, coms=coms,
                 frames=[Frame(6, eRL, epL), Frame(13, eRR, epR)], blocks=[blk],
                 spheres=np.array(spheres, np.float64), obstacles=obs, qref=qref, name="dual14_rel")


# ---- C3/C4: 36-DoF humanoid-like tree ------------------------------------
# joint index map (depth-first preorder)
H_BASE = list(range(0, 6))       # Px Py Pz Rz Ry Rx -> pelvis is link 5
H_LLEG = list(range(6, 12))      # hip z, hip x, hip y, knee y, ankle y, ankle x
H_RLEG = list(range(12, 18))
H_TORSO = [18, 19]               # torso z, torso y -> chest is link 19
H_LARM = list(range(20, 27))     # shoulder y, x, z, elbow y, wrist z, y, x
H_RARM = list(range(27, 34))
H_HEAD = [34, 35]                # neck z, neck y
H_PARENTS = ([-1, 0, 1, 2, 3, 4] + [5, 6, 7, 8, 9, 10] + [5, 12, 13, 14, 15, 16] + [5, 18] +
             [19, 20, 21, 22, 23, 24, 25] + [19, 27, 28, 29, 30, 31, 32] + [19, 34])
H_TYPES = [JOINT_PRI] * 3 + [JOINT_REV] * 33
H_AXES = ([0, 1, 2, 2, 1, 0] + [2, 0, 1, 1, 1, 0] * 2 + [2, 1] + [1, 0, 2, 1, 2, 1, 0] * 2 + [2, 1])
H_FRAMES = {"lfoot": 11, "rfoot": 17, "lhand": 26, "rhand": 33}


def humanoid_geometry(r):
    g = dict(
        hip_w=r.uniform(0.08, 0.12), hip_drop=r.uniform(0.05, 0.10),
        thigh=r.uniform(0.35, 0.45), shin=r.uniform(0.35, 0.45), foot_h=r.uniform(0.04, 0.08),
        torso_h=r.uniform(0.10, 0.20), chest=r.uniform(0.30, 0.40), shoulder_w=0.2,
        upper=r.uniform(0.25, 0.32), fore=r.uniform(0.25, 0.32), hand=r.uniform(0.05, 0.10),
        neck=r.uniform(0.03, 0.08), head=r.uniform(0.15, 0.25))
    return g


def _humanoid_body(config_id: int, n_slabs: int, bend: float, slab_x, slab_h) -> dict:
    """Joint tree, collision spheres, masses, the four end-effector frames, the nominal pose and the
    shelf-slab obstacles of the 36-DoF humanoid (shared by its two constraint sets)."""
    r = rng_for(config_id, 0)
    g = humanoid_geometry(r)
    I = np.eye(3)
    z = np.zeros(3)
    O = [z.copy() for _ in range(36)]
    O[6] = np.array([0.0, g["hip_w"], -g["hip_drop"]])
    O[12] = np.array([0.0, -g["hip_w"], -g["hip_drop"]])
    for base in (6, 12):
        O[base + 3] = np.array([0.0, 0.0, -g["thigh"]])
        O[base + 4] = np.array([0.0, 0.0, -g["shin"]])
    O[18] = np.array([0.0, 0.0, g["torso_h"]])
    O[20] = np.array([0.0, g["shoulder_w"], g["chest"]])
    O[27] = np.array([0.0, -g["shoulder_w"], g["chest"]])
    for base in (20, 27):
        O[base + 3] = np.array([0.0, 0.0, -g["upper"]])
        O[base + 4] = np.array([0.0, 0.0, -g["fore"]])
    O[34] = np.array([0.0, 0.0, g["chest"] + g["neck"]])
    joints = [Joint(H_PARENTS[j], H_TYPES[j], H_AXES[j], I, O[j]) for j in range(36)]

    # link sphere segments in each link frame (8 spheres per geometric link)
    short = 0.06
    seg = {5: (np.array([0.0, -g["hip_w"], -g["hip_drop"]]), np.array([0.0, g["hip_w"], -g["hip_drop"]]))}
    for base in (6, 12):
        seg[base + 0] = (z, np.array([0.0, 0.0, -short]))
        seg[base + 1] = (z, np.array([0.0, 0.0, -short]))
        seg[base + 2] = (z, np.array([0.0, 0.0, -g["thigh"]]))
        seg[base + 3] = (z, np.array([0.0, 0.0, -g["shin"]]))
        seg[base + 4] = (z, np.array([0.0, 0.0, -0.5 * g["foot_h"]]))
        seg[base + 5] = (np.array([-0.08, 0.0, -g["foot_h"] + 0.04]), np.array([0.12, 0.0, -g["foot_h"] + 0.04]))
    seg[18] = (z, np.array([0.0, 0.0, short]))
    seg[19] = (z, np.array([0.0, 0.0, g["chest"]]))
    for base in (20, 27):
        seg[base + 0] = (z, np.array([0.0, 0.0, -short]))
        seg[base + 1] = (z, np.array([0.0, 0.0, -short]))
        seg[base + 2] = (z, np.array([0.0, 0.0, -g["upper"]]))
        seg[base + 3] = (z, np.array([0.0, 0.0, -g["fore"]]))
        seg[base + 4] = (z, np.array([0.0, 0.0, -short]))
        seg[base + 5] = (z, np.array([0.0, 0.0, -short]))
        seg[base + 6] = (z, np.array([0.0, 0.0, -g["hand"]]))
    seg[34] = (z, np.array([0.0, 0.0, short]))
    seg[35] = (z, np.array([0.0, 0.0, g["head"]]))
    spheres = []
    for link in range(5, 36):
        s0, s1 = seg[link]
        spheres += _link_spheres(link, s1, 8, 0.04, start=s0)

    masses = np.zeros(36)
    coms = np.zeros((36, 3))
    for link in range(5, 36):
        s0, s1 = seg[link]
        coms[link] = 0.5 * (s0 + s1)
    masses[5] = r.uniform(8.0, 12.0)
    for base in (6, 12):
        mm = [r.uniform(0.5, 1.0), r.uniform(0.5, 1.0), r.uniform(4.0, 6.0), r.uniform(2.5, 4.0),
              r.uniform(0.3, 0.6), r.uniform(0.8, 1.2)]
        masses[base:base + 6] = mm if base == 6 else masses[6:12]
    masses[18] = r.uniform(1.0, 2.0)
    masses[19] = r.uniform(12.0, 18.0)
    for base in (20, 27):
        mm = [r.uniform(0.3, 0.6), r.uniform(0.3, 0.6), r.uniform(1.5, 2.5), r.uniform(1.0, 1.8),
              r.uniform(0.2, 0.4), r.uniform(0.2, 0.4), r.uniform(0.4, 0.7)]
        masses[base:base + 7] = mm if base == 20 else masses[20:27]
    masses[34] = r.uniform(0.3, 0.6)
    masses[35] = r.uniform(3.0, 4.5)

    # end-effector frames: sole centres and palms
    frames = [Frame(11, I, np.array([0.0, 0.0, -g["foot_h"]])),
              Frame(17, I, np.array([0.0, 0.0, -g["foot_h"]])),
              Frame(26, I, np.array([0.0, 0.0, -g["hand"]])),
              Frame(33, I, np.array([0.0, 0.0, -g["hand"]]))]
    qnom = humanoid_nominal(g, bend)
    ro = rng_for(config_id, 1)
    obs = []
    for _ in range(n_slabs):
        h = ro.uniform(*slab_h)
        x0 = ro.uniform(*slab_x)
        for iy in range(25):
            for ix in range(5):
                obs.append([x0 + 0.05 * ix, -0.6 + 0.05 * iy, h, 0.03])
    return dict(g=g, joints=joints, masses=masses, coms=coms, frames=frames, spheres=spheres, qnom=qnom, obs=obs)


def humanoid36_scene(config_id: int = 3, n_slabs: int = 4, bend: float = 0.3, slab_x=(0.35, 0.6),
                     slab_h=(0.2, 1.6)) -> Scene:
    """The 36-DoF humanoid with `n_slabs` shelf slabs of 25 x 5 obstacle spheres (r 0.03, pitch 0.05 m):
    front edge x0 ~ U[slab_x], height ~ U[slab_h]. The defaults keep the slabs in front of the robot;
    slab_x = (0.42, 0.5), slab_h = (1.0, 1.2) puts them in reach of the hands (a scene with collisions)."""
    hb = _humanoid_body(config_id, n_slabs, bend, slab_x, slab_h)
    g = hb["g"]
    # feet at fixed SE(3) poses on the floor, flat, hip-width apart
    bl = Block(BLK_POSE, fa=0, p=np.array([0.0, g["hip_w"], 0.0]))
    br = Block(BLK_POSE, fa=1, p=np.array([0.0, -g["hip_w"], 0.0]))
    # hands: fixed relative pose (the closed chain around the box), taken at the nominal pose
    bh = Block(BLK_REL, fa=2, fb=3, ref_from_qref=1)
    # CoM xy at the centroid of the support polygon (hull of the two 0.2 x 0.1 m soles, both centred on x = 0)
    bc = Block(BLK_COM, target=np.array([0.0, 0.0, 0.0]))

    return Scene(family=FAMILY_HUMANOID36, d=36, m=20, joints=hb["joints"], masses=hb["masses"], coms=hb["coms"],
                 frames=hb["frames"], blocks=[bl, br, bh, bc], spheres=np.array(hb["spheres"], np.float64),
                 obstacles=np.array(hb["obs"], np.float64), qref=hb["qnom"], name="humanoid36")


# sole contact patch of each foot in its sole frame (x forward, y left), for the support polygon
DIGIT_SOLE_X = (-0.03, 0.05)
DIGIT_SOLE_Y = (-0.03, 0.03)
DIGIT_TOE_OUT = 0.1  # foot yaw (rad), left +, right -


def digit36_scene(config_id: int = 5, n_slabs: int = 4, bend: float = 0.3, slab_x=(0.35, 0.6),
                  slab_h=(0.2, 1.6)) -> Scene:
    """The humanoid tree with the Digit constraint set of the paper's constraint figure: both feet at
    fixed poses (toed out by DIGIT_TOE_OUT), the hands' fixed relative pose, the CoM xy within the
    support polygon (the convex hull of the two sole contact patches at the feet's poses; the rows are
    the CoM minus its nearest point of the polygon, zero inside) and, per leg, a closed-linkage rod of
    fixed length between a point on the hip-roll link and a point on the shin (the length at the
    nominal pose)."""
    hb = _humanoid_body(config_id, n_slabs, bend, slab_x, slab_h)
    g = hb["g"]
    I = np.eye(3)
    frames = list(hb["frames"]) + [
        Frame(7, I, np.array([0.06, 0.0, -0.05])),    # 4: left hip rod end
        Frame(9, I, np.array([0.05, 0.0, -0.12])),    # 5: left tarsus rod end
        Frame(13, I, np.array([0.06, 0.0, -0.05])),   # 6: right hip rod end
        Frame(15, I, np.array([0.05, 0.0, -0.12]))]   # 7: right tarsus rod end
    Rl, Rr = rot_z(DIGIT_TOE_OUT), rot_z(-DIGIT_TOE_OUT)
    pl, pr = np.array([0.0, g["hip_w"], 0.0]), np.array([0.0, -g["hip_w"], 0.0])
    bl = Block(BLK_POSE, fa=0, R=Rl, p=pl)
    br = Block(BLK_POSE, fa=1, R=Rr, p=pr)
    bh = Block(BLK_REL, fa=2, fb=3, ref_from_qref=1)
    corners = np.array([[x, y, 0.0] for x in DIGIT_SOLE_X for y in DIGIT_SOLE_Y])
    patch = np.concatenate([(corners @ Rl.T + pl)[:, :2], (corners @ Rr.T + pr)[:, :2]])
    bc = hull_block(convex_hull_ccw(patch))
    dl = dist_block(4, 5, from_qref=True)
    dr = dist_block(6, 7, from_qref=True)
    return Scene(family=FAMILY_DIGIT36, d=36, m=22, joints=hb["joints"], masses=hb["masses"], coms=hb["coms"],
                 frames=frames, blocks=[bl, br, bh, bc, dl, dr], spheres=np.array(hb["spheres"], np.float64),
                 obstacles=np.array(hb["obs"], np.float64), qref=hb["qnom"], name="digit36")


def humanoid_nominal(g, bend=0.3):
    """A standing pose with bent knees and the arms forward holding a box (input recipe, approximate)."""
    q = np.zeros(36)
    # pelvis height for a symmetric knee bend (hip pitch -b, knee 2b, ankle -b), feet flat on the floor
    q[2] = g["hip_drop"] + (g["thigh"] + g["shin"]) * math.cos(bend) + g["foot_h"]
    for base in (6, 12):
        q[base + 2] = -bend
        q[base + 3] = 2 * bend
        q[base + 4] = -bend
    for base in (20, 27):
        q[base + 0] = -0.5
        q[base + 3] = -0.9
    return q


def humanoid_noise_sigma():
    s = np.full(36, 0.1)
    s[0:3] = 0.02
    s[3:6] = 0.05
    return s


# ---- geodesic endpoint sampling for C2-C4 ---------------------------------
def raw_endpoints(scene: Scene, config_id: int, n_geo: int, sigma):
    """Raw geodesic endpoints q_ref + N(0, sigma^2), shape [n_geo, 2, d] (projected later by whichever
    implementation consumes them)."""
    r = rng_for(config_id, 2)
    sig = np.broadcast_to(np.asarray(sigma, np.float64), (scene.d,))
    e = scene.qref[None, None, :] + r.standard_normal((n_geo, 2, scene.d)) * sig[None, None, :]
    return e


def geodesic_lengths(config_id: int, n_geo: int, lo: int, hi: int):
    r = rng_for(config_id, 4)
    L = r.integers(lo, hi + 1, n_geo)
    offs = np.zeros(n_geo + 1, np.int32)
    offs[1:] = np.cumsum(L)
    return offs


def make_config(name: str, small: bool = False):
    """The scenes and raw workloads of the five benchmark configurations.

    Returns a dict: scene, tol, max_iter, and either q (final raw batch) or endpoints + geo_offsets
    (batches built by projecting endpoints, then interpolating interior points)."""
    if name == "c0":
        sc = sphere_scene(0)
        q, offs = sphere_workload(0, n_seg=64 if small else 1024)
        return dict(name=name, scene=sc, tol=1e-6, max_iter=50, q=q, geo_offsets=offs)
    if name == "c1":
        sc = arm7_axis_scene(1)
        q, offs = arm7_workload(1, n_seg=64 if small else 4096)
        return dict(name=name, scene=sc, tol=1e-6, max_iter=30, q=q, geo_offsets=offs)
    if name == "c2":
        sc = dual14_rel_scene(2)
        n_geo = 64 if small else 16384
        return dict(name=name, scene=sc, tol=1e-6, max_iter=30,
                    endpoints=raw_endpoints(sc, 2, n_geo, 0.1),
                    geo_offsets=geodesic_lengths(2, n_geo, 4, 128))
    if name == "c3":
        sc = humanoid36_scene(3)
        n_geo = 32 if small else 2048
        return dict(name=name, scene=sc, tol=1e-6, max_iter=40,
                    endpoints=raw_endpoints(sc, 3, n_geo, humanoid_noise_sigma()),
                    geo_offsets=np.arange(n_geo + 1, dtype=np.int32) * 32)
    if name == "c3near":
        # the humanoid batch recipe with the shelf slabs moved into reach of the hands (a test scene
        # in which most projected configurations collide); 256 geodesics = 8,192 configurations
        sc = humanoid36_scene(3, slab_x=(0.42, 0.5), slab_h=(1.0, 1.2))
        n_geo = 32 if small else 256
        return dict(name=name, scene=sc, tol=1e-6, max_iter=40,
                    endpoints=raw_endpoints(sc, 3, n_geo, humanoid_noise_sigma()),
                    geo_offsets=np.arange(n_geo + 1, dtype=np.int32) * 32)
    if name == "c4":
        sc = humanoid36_scene(3)
        n_geo = 32 if small else 2048
        return dict(name=name, scene=sc, tol=1e-6, max_iter=40,
                    endpoints=raw_endpoints(sc, 4, n_geo, humanoid_noise_sigma()),
                    geo_offsets=geodesic_lengths(4, n_geo, 8, 64))
    if name == "c5":
        # the Digit constraint set on the humanoid (closed linkages, CoM within the support polygon)
        sc = digit36_scene(5)
        n_geo = 32 if small else 2048
        return dict(name=name, scene=sc, tol=1e-6, max_iter=40,
                    endpoints=raw_endpoints(sc, 5, n_geo, humanoid_noise_sigma()),
                    geo_offsets=np.arange(n_geo + 1, dtype=np.int32) * 32)
    if name == "c6":
        # the 7-DoF arm with a bounded TSR: geodesics between projected endpoints q_ref + N(0, 0.2^2)
        sc = arm7_tsr_scene(6)
        n_geo = 64 if small else 4096
        return dict(name=name, scene=sc, tol=1e-6, max_iter=30,
                    endpoints=raw_endpoints(sc, 6, n_geo, 0.2),
                    geo_offsets=np.arange(n_geo + 1, dtype=np.int32) * 32)
    raise ValueError(name)


# ---- ConstrainedExtend workloads --------------------------------------------
# Extension parameters per configuration: range r, resolution delta, particles n, particle spread
# sigma (the paper tunes r and sigma per robot and does not list the values; these keep the
# steer point within a few Newton steps of the manifold).
EXTEND_PARAMS = {
    "c0": dict(r=0.5, delta=0.05, n=8, sigma=0.1),
    "c1": dict(r=0.4, delta=0.05, n=8, sigma=0.05),
    "c3": dict(r=0.3, delta=0.02, n=8, sigma=0.05),
}


def extend_workload(name: str, E: int):
    """Raw inputs of E extensions on configuration `name`: starts [E, d] (raw: the consumer projects
    them onto the manifold first, except on the sphere where they are unit vectors already),
    targets [E, d] (ambient points, like RRT's random samples) and the particle draws eps [E, n]
    ~ N(0, sigma^2). Returns dict(scene, starts, targets, eps, starts_on_manifold, **EXTEND_PARAMS)."""
    prm = EXTEND_PARAMS[name]
    cid = CONFIG_IDS[name]
    r5 = rng_for(cid, 5)
    if name == "c0":
        sc = sphere_scene(0)
        r2 = rng_for(cid, 2)
        starts = _uniform_sphere_points(r2, E)
        dirs = _uniform_sphere_points(r2, E)
        targets = starts + dirs * r2.uniform(0.2, 1.5, (E, 1))
        on = True
    elif name == "c1":
        sc = arm7_axis_scene(1)
        r2 = rng_for(cid, 2)
        starts = r2.uniform(-np.pi, np.pi, (E, 7))
        targets = starts + r2.normal(0.0, 0.5, (E, 7))
        on = False
    elif name == "c3":
        sc = humanoid36_scene(3)
        ends = raw_endpoints(sc, 3, E, humanoid_noise_sigma())
        starts, targets = ends[:, 0], ends[:, 1]
        on = False
    else:
        raise ValueError(name)
    eps = r5.normal(0.0, prm["sigma"], (E, prm["n"]))
    return dict(name=name, scene=sc, starts=np.ascontiguousarray(starts), targets=np.ascontiguousarray(targets),
                eps=eps, starts_on_manifold=on, tol=1e-6, max_iter={"c0": 50, "c1": 30, "c3": 40}[name], **prm)
