"""Pins of the FP64 oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: a closed form,
a textbook routine reached by a different route, an identity, or brute force.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2604_13323_amd import scenes as S

CONV, MAXIT, SING, DIV, NONF = range(5)


def prob(scene):
    import oracle
    return oracle.Problem(scene.to_blob())


# ---------------------------------------------------------------- sphere
def test_sphere_closed_form_and_heron_counts(oracle_mod):
    """Min-norm Newton on ||q||^2 - 1 is radial: r -> (r + 1/r)/2 (Heron), fixed point q/||q||.
    Step counts to |r^2 - 1| < 1e-6, worked out in exact rationals: 0.9->3, 0.5->4, 0.1->7, 0.01->10, 3->5."""
    P = prob(S.sphere_scene(0))
    rng = np.random.default_rng(7)
    for r0, k in [(0.9, 3), (0.5, 4), (0.1, 7), (0.01, 10), (3.0, 5)]:
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        qo, st, it, rs = P.project((r0 * u)[None], tol=1e-6, max_iter=50)
        assert st[0] == CONV and it[0] == k, (r0, st[0], it[0])
        np.testing.assert_allclose(qo[0], u, atol=1e-6)
        assert rs[0] < 1e-6


def test_sphere_heron_counts_match_golden_fixture(oracle_mod):
    """The stored table (tests/golden/heron_counts.txt, written from the recurrence in exact
    rationals by tests/golden/make_golden.py) against the oracle."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "heron_counts.txt")
    P = prob(S.sphere_scene(0))
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    u = np.array([0.6, 0.0, 0.8])
    for r0, k in rows:
        qo, st, it, rs = P.project((float(r0) * u)[None], tol=1e-6, max_iter=50)
        assert st[0] == CONV and it[0] == int(k), (r0, it[0], k)


def test_sphere_random_batch_matches_normalisation(oracle_mod):
    P = prob(S.sphere_scene(0))
    q, _ = S.sphere_workload(0, n_seg=32)
    qo, st, it, rs = P.project(q, tol=1e-12, max_iter=60)
    assert np.all(st == CONV)
    np.testing.assert_allclose(qo, q / np.linalg.norm(q, axis=1, keepdims=True), atol=1e-12)


def test_forced_statuses(oracle_mod):
    P = prob(S.sphere_scene(0))
    qo, st, it, rs = P.project(np.zeros((1, 3)), tol=1e-6, max_iter=50)
    assert st[0] == SING and it[0] == 0
    qo, st, it, rs = P.project(np.array([[np.nan, 0.0, 1.0]]), tol=1e-6, max_iter=50)
    assert st[0] == NONF
    qo, st, it, rs = P.project(np.array([[0.1, 0.0, 0.0]]), tol=1e-6, max_iter=1)
    assert st[0] == MAXIT and it[0] == 1
    # from r = 0.1 the first step has length 4.95 > 1: divergence exit, iterate untouched
    qo, st, it, rs = P.project(np.array([[0.1, 0.0, 0.0]]), tol=1e-6, max_iter=50, max_step=1.0)
    assert st[0] == DIV and it[0] == 0
    np.testing.assert_array_equal(qo[0], [0.1, 0.0, 0.0])
    # an input already on the manifold takes zero steps
    qo, st, it, rs = P.project(np.array([[0.0, 0.6, 0.8]]), tol=1e-6, max_iter=50)
    assert st[0] == CONV and it[0] == 0


# ---------------------------------------------------------------- linear
def test_linear_one_step_is_least_norm_correction(oracle_mod):
    """F = A q - b: one min-norm Newton step gives q - A^+ (A q - b), the lstsq least-norm correction."""
    rng = np.random.default_rng(3)
    for (m, d) in [(1, 3), (2, 5), (3, 7), (4, 8)]:
        A = rng.standard_normal((m, d))
        b = rng.standard_normal(m)
        P = prob(S.linear_scene(A, b))
        q0 = rng.standard_normal((5, d))
        qo, st, it, rs = P.project(q0, tol=1e-9, max_iter=10)
        assert np.all(st == CONV) and np.all(it == 1)
        for i in range(5):
            corr = np.linalg.lstsq(A, A @ q0[i] - b, rcond=None)[0]
            np.testing.assert_allclose(qo[i], q0[i] - corr, atol=1e-12)


def test_linear_damped_step(oracle_mod):
    """lambda > 0: step = A^T (A A^T + lambda I)^-1 (A q - b), here from the normal-equation form."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((2, 5))
    b = rng.standard_normal(2)
    P = prob(S.linear_scene(A, b))
    q0 = rng.standard_normal((1, 5))
    lam, alpha = 0.3, 0.7
    qo, st, it, rs = P.project(q0, tol=1e-30, max_iter=1, alpha=alpha, lam=lam)
    assert st[0] == MAXIT and it[0] == 1
    step = alpha * A.T @ np.linalg.solve(A @ A.T + lam * np.eye(2), A @ q0[0] - b)
    np.testing.assert_allclose(qo[0], q0[0] - step, atol=1e-12)


def test_damped_step_equals_the_outer_pseudo_inverse_form(oracle_mod):
    """Alg. 2 offers the step with the inner pseudo-inverse, J^T (J J^T + lambda I)^-1 d, or the outer one,
    (J^T J + lambda I)^-1 J^T d. For lambda > 0 they are the same vector (push-through identity), so the
    library's inner form also gives the outer form's step; here the oracle's damped step is compared with the
    d x d outer system solved directly."""
    rng = np.random.default_rng(14)
    A = rng.standard_normal((3, 6))
    b = rng.standard_normal(3)
    P = prob(S.linear_scene(A, b))
    q0 = rng.standard_normal((1, 6))
    lam = 0.05
    qo, _, _, _ = P.project(q0, tol=1e-30, max_iter=1, lam=lam)
    outer = np.linalg.solve(A.T @ A + lam * np.eye(6), A.T @ (A @ q0[0] - b))
    np.testing.assert_allclose(qo[0], q0[0] - outer, atol=1e-12)


def test_linear_vjp_is_pinv_projector(oracle_mod):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((3, 7))
    P = prob(S.linear_scene(A, rng.standard_normal(3)))
    q = rng.standard_normal((4, 7))
    g = rng.standard_normal((4, 7))
    gi, kap = P.vjp(q, g)
    Pn = np.eye(7) - np.linalg.pinv(A) @ A
    np.testing.assert_allclose(gi, g @ Pn.T, atol=1e-12)
    sv = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(kap, (sv[0] / sv[-1]) ** 2, rtol=1e-10)


# ---------------------------------------------------------------- planar 2R arm
def _ik_2r(l1, l2, x, y):
    c2 = (x * x + y * y - l1 * l1 - l2 * l2) / (2 * l1 * l2)
    sols = []
    for s in (+1, -1):
        q2 = s * math.acos(c2)
        q1 = math.atan2(y, x) - math.atan2(l2 * math.sin(q2), l1 + l2 * math.cos(q2))
        sols.append((q1, q2))
    return sols


def _wrap(a):
    return (a + math.pi) % (2 * math.pi) - math.pi


def test_planar_2r_matches_analytic_ik(oracle_mod):
    rng = np.random.default_rng(11)
    l1, l2 = 0.7, 0.5
    for _ in range(20):
        rad = rng.uniform(0.3, 1.1)
        ang = rng.uniform(-math.pi, math.pi)
        x, y = rad * math.cos(ang), rad * math.sin(ang)
        P = prob(S.planar2_scene(l1, l2, (x, y)))
        sols = _ik_2r(l1, l2, x, y)
        # start near one branch
        q1, q2 = sols[rng.integers(2)]
        q0 = np.array([[q1 + rng.normal(0, 0.15), q2 + rng.normal(0, 0.15)]])
        qo, st, it, rs = P.project(q0, tol=1e-12, max_iter=50)
        assert st[0] == CONV
        err = min(max(abs(_wrap(qo[0, 0] - a)), abs(_wrap(qo[0, 1] - b))) for a, b in sols)
        assert err < 1e-9, err


def test_planar_2r_unreachable(oracle_mod):
    P = prob(S.planar2_scene(0.7, 0.5, (2.0, 0.5)))
    qo, st, it, rs = P.project(np.array([[0.1, 0.2]]), tol=1e-6, max_iter=40)
    assert st[0] in (MAXIT, SING)


def test_planar_tip_residual_closed_form(oracle_mod):
    l1, l2, tx, ty = 0.7, 0.5, 0.3, -0.2
    P = prob(S.planar2_scene(l1, l2, (tx, ty)))
    rng = np.random.default_rng(2)
    q = rng.uniform(-3, 3, (10, 2))
    F = P.residual(q)
    x = l1 * np.cos(q[:, 0]) + l2 * np.cos(q[:, 0] + q[:, 1])
    y = l1 * np.sin(q[:, 0]) + l2 * np.sin(q[:, 0] + q[:, 1])
    np.testing.assert_allclose(F, np.stack([x - tx, y - ty], 1), atol=1e-14)


# ---------------------------------------------------------------- kinematics
def _dh(theta, d, a, alpha):
    ct, st, ca, sa = math.cos(theta), math.sin(theta), math.cos(alpha), math.sin(alpha)
    return np.array([[ct, -st * ca, st * sa, a * ct],
                     [st, ct * ca, -ct * sa, a * st],
                     [0, sa, ca, d],
                     [0, 0, 0, 1.0]])


def test_dh_arm_fk_matches_textbook_dh_product(oracle_mod):
    """The origin/axis form of the generator + the oracle's FK equal the standard DH product
    T = prod_i Rz(theta_i) Tz(d_i) Tx(a_i) Rx(alpha_i) at the end-effector."""
    sc = S.arm7_axis_scene(1)
    P = prob(sc)
    r = S.rng_for(1, 0)
    a, d, alpha = S._dh_params(r)
    rng = np.random.default_rng(0)
    for _ in range(10):
        q = rng.uniform(-math.pi, math.pi, 7)
        T = np.eye(4)
        for i in range(7):
            T = T @ _dh(q[i], d[i], a[i], alpha[i])
        ee = P.frame_poses(q)[0]
        np.testing.assert_allclose(ee[:9].reshape(3, 3), T[:3, :3], atol=1e-13)
        np.testing.assert_allclose(ee[9:], T[:3, 3], atol=1e-13)


def test_axis_residual_is_ee_z_xy(oracle_mod):
    sc = S.arm7_axis_scene(1)
    P = prob(sc)
    r = S.rng_for(1, 0)
    a, d, alpha = S._dh_params(r)
    q = np.random.default_rng(1).uniform(-3, 3, (6, 7))
    F = P.residual(q)
    for i in range(6):
        T = np.eye(4)
        for k in range(7):
            T = T @ _dh(q[i, k], d[k], a[k], alpha[k])
        np.testing.assert_allclose(F[i], T[:2, 2], atol=1e-13)


def test_humanoid_rigid_links_and_rotations(oracle_mod):
    """Rigid-body invariants: every link rotation is orthonormal with det 1, and the distance between a
    joint's origin and its parent's origin equals the fixed origin offset at any configuration."""
    sc = S.humanoid36_scene(3)
    P = prob(sc)
    rng = np.random.default_rng(5)
    for _ in range(5):
        q = sc.qref + rng.normal(0, 0.5, 36)
        L = P.link_frames(q)
        for j in range(36):
            R = L[j, :9].reshape(3, 3)
            np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-13)
            assert abs(np.linalg.det(R) - 1) < 1e-13
            par = sc.joints[j].parent
            if par >= 0 and sc.joints[j].jtype == S.JOINT_REV:
                np.testing.assert_allclose(np.linalg.norm(L[j, 9:] - L[par, 9:]),
                                           np.linalg.norm(sc.joints[j].p), atol=1e-13)


def test_humanoid_zero_pose_closed_form(oracle_mod):
    """At q = 0 every frame is axis-aligned and the sole centre sits at the summed offsets."""
    sc = S.humanoid36_scene(3)
    P = prob(sc)
    fr = P.frame_poses(np.zeros(36))
    off = sum(sc.joints[j].p for j in range(6, 12)) + sc.frames[0].p
    np.testing.assert_allclose(fr[0, 9:], off, atol=1e-14)
    np.testing.assert_allclose(fr[0, :9].reshape(3, 3), np.eye(3), atol=1e-14)
    # base prismatic joints translate the whole robot
    q = np.zeros(36)
    q[:3] = [0.3, -0.2, 0.9]
    np.testing.assert_allclose(P.frame_poses(q)[0, 9:], off + q[:3], atol=1e-14)


def test_single_joint_rotation_is_rodrigues(oracle_mod):
    """Turning one revolute joint by t rotates every downstream frame about that joint's world axis
    through its origin (checked with scipy's rotation-vector map)."""
    sc = S.humanoid36_scene(3)
    P = prob(sc)
    rng = np.random.default_rng(9)
    q = sc.qref + rng.normal(0, 0.3, 36)
    for j in (8, 21, 35):
        t = 0.37
        L0 = P.link_frames(q)
        q1 = q.copy()
        q1[j] += t
        L1 = P.link_frames(q1)
        ax = sc.joints[j].axis
        zj = L0[j, :9].reshape(3, 3)[:, ax]
        oj = L0[j, 9:]
        Rw = Rotation.from_rotvec(zj * t).as_matrix()
        sub = {j}
        for k in range(j + 1, 36):
            if sc.joints[k].parent in sub:
                sub.add(k)
        for k in range(36):
            if k not in sub:
                np.testing.assert_allclose(L1[k], L0[k], atol=0)
                continue
            np.testing.assert_allclose(L1[k, 9:], oj + Rw @ (L0[k, 9:] - oj), atol=1e-12)
            np.testing.assert_allclose(L1[k, :9].reshape(3, 3), Rw @ L0[k, :9].reshape(3, 3), atol=1e-12)


def test_com_of_prismatic_chain_closed_form(oracle_mod):
    """Two prismatic joints (x then y) carrying point masses: CoM xy = q shifted by the mass-weighted offsets."""
    I = np.eye(3)
    joints = [S.Joint(-1, S.JOINT_PRI, 0, I, np.zeros(3)), S.Joint(0, S.JOINT_PRI, 1, I, np.zeros(3))]
    masses = np.array([2.0, 3.0])
    coms = np.array([[0.1, 0.0, 0.0], [0.0, -0.4, 0.5]])
    sc = S.Scene(family=S.FAMILY_LINEAR, d=2, m=2, joints=joints, masses=masses, coms=coms,
                 blocks=[S.Block(S.BLK_COM, target=np.array([0.05, 0.02, 0.0]))],
                 spheres=np.zeros((0, 5)), obstacles=np.zeros((0, 4)))
    P = prob(sc)
    q = np.array([[0.3, 0.7], [-1.0, 2.0]])
    F = P.residual(q)
    cx = (2 * (q[:, 0] + 0.1) + 3 * q[:, 0]) / 5
    cy = (3 * (q[:, 1] - 0.4)) / 5
    np.testing.assert_allclose(F, np.stack([cx - 0.05, cy - 0.02], 1), atol=1e-15)


# ---------------------------------------------------------------- SO(3) log and pose errors
def test_so3_log_inverts_exp(oracle_mod):
    import oracle
    rng = np.random.default_rng(1)
    for ang in [1e-9, 1e-6, 5e-5, 2e-4, 1e-2, 0.5, 1.5, 2.5, 3.0]:
        for _ in range(5):
            ax = rng.standard_normal(3)
            w = ax / np.linalg.norm(ax) * ang
            R = Rotation.from_rotvec(w).as_matrix()
            np.testing.assert_allclose(oracle.so3_log(R), w, atol=1e-12 * max(1.0, ang / (math.pi - ang)))
    np.testing.assert_allclose(oracle.so3_log(np.eye(3)), np.zeros(3), atol=0)


def test_pose_rotation_rows_single_joint(oracle_mod):
    """One revolute joint about z and a full 6-row pose block: rows = (R_ref^T p, (0, 0, q - theta_ref))."""
    I = np.eye(3)
    th = 0.4
    Rr = Rotation.from_rotvec([0, 0, th]).as_matrix()
    # joint 0 carries the frame; joints 1..5 hang below it and do not move it (m = 6 needs d >= 6)
    joints = [S.Joint(-1, S.JOINT_REV, 2, I, np.zeros(3))] + \
        [S.Joint(k, S.JOINT_REV, 2, I, np.array([0.5, 0, 0])) for k in range(5)]
    blk = S.Block(S.BLK_POSE, fa=0, mask=0x3F, R=Rr, p=np.zeros(3))
    sc = S.Scene(family=S.FAMILY_PLANAR2, d=6, m=6, joints=joints, masses=np.ones(6), coms=np.zeros((6, 3)),
                 frames=[S.Frame(0, I, np.zeros(3))], blocks=[blk], spheres=np.zeros((0, 5)),
                 obstacles=np.zeros((0, 4)))
    P = prob(sc)
    for q0 in (-1.0, 0.0, 0.4, 1.3):
        F = P.residual(np.array([[q0, 0.7, 0.1, 0.2, 0.3, 0.4]]))[0]
        np.testing.assert_allclose(F, [0, 0, 0, 0, 0, q0 - th], atol=1e-14)


def test_relative_pose_zero_at_reference_and_base_invariant(oracle_mod):
    sc = S.dual14_rel_scene(2)
    P = prob(sc)
    assert np.max(np.abs(P.residual(sc.qref[None]))) < 1e-14
    # Eq. 2 is invariant to a common motion of both arms: move both bases by the same rigid transform
    I = np.eye(3)
    rng = np.random.default_rng(3)
    q = sc.qref + rng.normal(0, 0.2, 14)
    F0 = P.residual(q[None])[0]
    Rb = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    pb = np.array([0.4, 0.1, -0.3])
    joints = [S.Joint(-1, S.JOINT_REV, 2, Rb, pb)]  # a shared root joint holding both arms
    for j in sc.joints:
        parent = 0 if j.parent < 0 else j.parent + 1
        joints.append(S.Joint(parent, j.jtype, j.axis, j.R, j.p))
    frames = [S.Frame(f.link + 1, f.R, f.p) for f in sc.frames]
    sc2 = S.Scene(family=S.FAMILY_DUAL14_REL, d=15, m=6, joints=joints, masses=np.ones(15),
                  coms=np.zeros((15, 3)), frames=frames, blocks=sc.blocks, spheres=np.zeros((0, 5)),
                  obstacles=np.zeros((0, 4)), qref=np.concatenate([[0.0], sc.qref]))
    P2 = prob(sc2)
    for t in (0.0, 0.8, -2.0):
        np.testing.assert_allclose(P2.residual(np.concatenate([[t], q])[None])[0], F0, atol=1e-12)


# ---------------------------------------------------------------- Jacobian vs finite differences
@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3"])
def test_dual_jacobian_matches_central_fd(oracle_mod, name):
    cfg = S.make_config(name, small=True)
    sc = cfg["scene"]
    P = prob(sc)
    rng = np.random.default_rng(1)
    if sc.qref is not None:
        q = sc.qref[None] + rng.normal(0, 0.2, (4, sc.d))
    else:
        q = cfg["q"][:4]
    J = P.jacobian(q)
    h = 1e-6
    for j in range(sc.d):
        e = np.zeros(sc.d)
        e[j] = h
        fd = (P.residual(q + e) - P.residual(q - e)) / (2 * h)
        np.testing.assert_allclose(J[:, :, j], fd, atol=2e-8, rtol=1e-6)


# ---------------------------------------------------------------- VJP identities
@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3"])
def test_vjp_tangent_projector_identities(oracle_mod, name):
    cfg = S.make_config(name, small=True)
    sc = cfg["scene"]
    P = prob(sc)
    rng = np.random.default_rng(2)
    q0 = sc.qref[None] + rng.normal(0, 0.05, (6, sc.d)) if sc.qref is not None else cfg["q"][:6]
    qs, st, it, rs = P.project(q0, tol=1e-12, max_iter=100)
    assert np.all(st == CONV)
    g = rng.standard_normal(qs.shape)
    h = rng.standard_normal(qs.shape)
    gi, kap = P.vjp(qs, g, st)
    J = P.jacobian(qs)
    # J (I - J^+ J) g = 0
    assert np.max(np.abs(np.einsum("nmd,nd->nm", J, gi))) < 1e-11 * max(1.0, np.abs(J).max())
    # idempotent and symmetric
    gii, _ = P.vjp(qs, gi, st)
    np.testing.assert_allclose(gii, gi, atol=1e-12)
    hi, _ = P.vjp(qs, h, st)
    np.testing.assert_allclose(np.sum(gi * h, 1), np.sum(g * hi, 1), atol=1e-11)
    # non-converged configurations get zero
    st2 = st.copy()
    st2[0] = MAXIT
    gz, _ = P.vjp(qs, g, st2)
    assert np.all(gz[0] == 0)


def test_vjp_sphere_closed_form(oracle_mod):
    P = prob(S.sphere_scene(0))
    rng = np.random.default_rng(8)
    u = rng.standard_normal((10, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    g = rng.standard_normal((10, 3))
    gi, _ = P.vjp(u, g, np.zeros(10, np.int8))
    np.testing.assert_allclose(gi, g - np.sum(g * u, 1, keepdims=True) * u, atol=1e-14)


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_vjp_equals_fd_of_projection_on_manifold(oracle_mod, name):
    """At an on-manifold input, d P(q0)/d q0 = I - J^+ J exactly: FP64 central differences of the
    Newton projection (run to ||F|| < 1e-13) reproduce the VJP."""
    cfg = S.make_config(name, small=True)
    sc = cfg["scene"]
    P = prob(sc)
    rng = np.random.default_rng(4)
    q0 = sc.qref[None] + rng.normal(0, 0.05, (2, sc.d)) if sc.qref is not None else cfg["q"][:2]
    qs, st, it, rs = P.project(q0, tol=1e-13, max_iter=100)
    assert np.all(st == CONV)
    h = 1e-6
    for c in range(2):
        g = rng.standard_normal(sc.d)
        Jfd = np.zeros((sc.d, sc.d))
        for j in range(sc.d):
            e = np.zeros(sc.d)
            e[j] = h
            qp = P.project((qs[c] + e)[None], tol=1e-13, max_iter=100)[0][0]
            qm = P.project((qs[c] - e)[None], tol=1e-13, max_iter=100)[0][0]
            Jfd[:, j] = (qp - qm) / (2 * h)
        gi, _ = P.vjp(qs[c:c + 1], g[None], st[c:c + 1])
        np.testing.assert_allclose(gi[0], Jfd.T @ g, atol=1e-6 * np.linalg.norm(g))


# ---------------------------------------------------------------- collision
def test_collision_point_robot_margins(oracle_mod):
    """Point robot (r = 0) vs one obstacle sphere: strict overlap test, exact signed distance."""
    sc = S.sphere_scene(0)
    sc.obstacles = np.array([[0.0, 0.0, 0.0, 0.5]])
    P = prob(sc)
    u = np.array([0.6, 0.0, 0.8])
    q = np.stack([u * (0.5 - 2e-5), u * (0.5 + 2e-5), u * 0.5, u * 0.1])
    v, sd = P.check(q)
    np.testing.assert_array_equal(v, [1, 0, 0, 1])
    np.testing.assert_allclose(sd, [-2e-5, 2e-5, 0.0, -0.4], atol=1e-15)


def test_collision_brute_force_matches_scipy_distances(oracle_mod):
    """Robot sphere centres from the link frames vs obstacles, checked against scipy's cdist."""
    from scipy.spatial.distance import cdist
    sc = S.arm7_axis_scene(1)
    P = prob(sc)
    rng = np.random.default_rng(6)
    q = rng.uniform(-3, 3, (20, 7))
    v, sd = P.check(q)
    for i in range(20):
        L = P.link_frames(q[i])
        cen = np.array([L[int(s[0]), :9].reshape(3, 3) @ s[1:4] + L[int(s[0]), 9:] for s in sc.spheres])
        D = cdist(cen, sc.obstacles[:, :3]) - (sc.spheres[:, 4][:, None] + sc.obstacles[:, 3][None, :])
        assert v[i] == int(D.min() < 0)
        np.testing.assert_allclose(sd[i], D.min(), atol=1e-13)


def test_path_length_gradient_fd(oracle_mod):
    import oracle
    rng = np.random.default_rng(0)
    q = rng.standard_normal((12, 4))
    offs = np.array([0, 5, 12], np.int32)
    L, g = oracle.path_length(q, offs)
    ref = sum(np.linalg.norm(np.diff(q[a:b], axis=0), axis=1).sum() for a, b in [(0, 5), (5, 12)])
    assert abs(L - ref) < 1e-12
    h = 1e-6
    for i in range(12):
        for j in range(4):
            e = np.zeros_like(q)
            e[i, j] = h
            fd = (oracle.path_length(q + e, offs)[0] - oracle.path_length(q - e, offs)[0]) / (2 * h)
            assert abs(fd - g[i, j]) < 1e-7


def test_com_revolute_closed_form(oracle_mod):
    """A revolute joint about z with a point mass at (a, 0, h) and a fixed base mass: CoM rotates with q."""
    I = np.eye(3)
    joints = [S.Joint(-1, S.JOINT_PRI, 2, I, np.zeros(3)), S.Joint(0, S.JOINT_REV, 2, I, np.array([0.2, 0.0, 0.0]))]
    masses = np.array([1.0, 3.0])
    coms = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.1]])
    sc = S.Scene(family=S.FAMILY_LINEAR, d=2, m=2, joints=joints, masses=masses, coms=coms,
                 blocks=[S.Block(S.BLK_COM)], spheres=np.zeros((0, 5)), obstacles=np.zeros((0, 4)))
    P = prob(sc)
    for q1 in (-2.0, 0.3, 1.1):
        F = P.residual(np.array([[0.0, q1]]))[0]
        cx = (3 * (0.2 + 0.5 * math.cos(q1))) / 4
        cy = (3 * (0.5 * math.sin(q1))) / 4
        np.testing.assert_allclose(F, [cx, cy], atol=1e-15)


def test_relative_pose_frame_order_closed_form(oracle_mod):
    """Eq. 2 with T_ref = I: frame a on a revolute-z link, frame b on a prismatic-x link.
    T_a^-1 T_b = (Rz(-q0), Rz(-q0) (q1, 0, 0)), so rows = (q1 cos q0, -q1 sin q0, 0, 0, 0, -q0)."""
    I = np.eye(3)
    joints = [S.Joint(-1, S.JOINT_REV, 2, I, np.zeros(3)), S.Joint(-1, S.JOINT_PRI, 0, I, np.zeros(3))] + \
        [S.Joint(-1, S.JOINT_PRI, 1, I, np.zeros(3)) for _ in range(4)]
    blk = S.Block(S.BLK_REL, fa=0, fb=1)
    sc = S.Scene(family=S.FAMILY_DUAL14_REL, d=6, m=6, joints=joints, masses=np.ones(6), coms=np.zeros((6, 3)),
                 frames=[S.Frame(0, I, np.zeros(3)), S.Frame(1, I, np.zeros(3))], blocks=[blk],
                 spheres=np.zeros((0, 5)), obstacles=np.zeros((0, 4)))
    P = prob(sc)
    for q0, q1 in [(0.3, 0.7), (-1.2, 0.25), (2.0, -0.5)]:
        F = P.residual(np.array([[q0, q1, 0, 0, 0, 0]]))[0]
        np.testing.assert_allclose(F, [q1 * math.cos(q0), -q1 * math.sin(q0), 0, 0, 0, -q0], atol=1e-14)


def test_pose_translation_rows_rotated_target(oracle_mod):
    """Eq. 1 translation rows are expressed in the target frame: R_ref^T (p - p_ref)."""
    I = np.eye(3)
    th = 0.4
    Rr = Rotation.from_rotvec([0, 0, th]).as_matrix()
    joints = [S.Joint(-1, S.JOINT_REV, 2, I, np.zeros(3))] + \
        [S.Joint(k, S.JOINT_REV, 2, I, np.array([0.5, 0, 0])) for k in range(5)]
    pref = np.array([0.05, -0.02, 0.0])
    blk = S.Block(S.BLK_POSE, fa=0, mask=0x3F, R=Rr, p=pref)
    sc = S.Scene(family=S.FAMILY_PLANAR2, d=6, m=6, joints=joints, masses=np.ones(6), coms=np.zeros((6, 3)),
                 frames=[S.Frame(0, I, np.array([0.3, 0.0, 0.0]))], blocks=[blk], spheres=np.zeros((0, 5)),
                 obstacles=np.zeros((0, 4)))
    P = prob(sc)
    for q0 in (-1.0, 0.4, 1.3):
        F = P.residual(np.array([[q0, 0, 0, 0, 0, 0]]))[0]
        p = np.array([0.3 * math.cos(q0), 0.3 * math.sin(q0), 0.0])
        np.testing.assert_allclose(F[:3], Rr.T @ (p - pref), atol=1e-14)
        np.testing.assert_allclose(F[3:], [0, 0, q0 - th], atol=1e-14)


# ---------------------------------------------------------------- cyclic mode (Sec. IV-C, Alg. 2)
def _two_sphere_block_scene():
    import dataclasses
    sc = S.sphere_scene(0)
    return dataclasses.replace(sc, m=2, blocks=[S.Block(S.BLK_SPHERE), S.Block(S.BLK_SPHERE)])


def test_cyclic_two_sphere_blocks_is_two_heron_steps_per_iteration(oracle_mod):
    """Two copies of ||q||^2 - 1 as separate blocks: each block's min-norm step is one Heron step
    r -> (r + 1/r)/2 on the radius, so a cyclic iteration takes two of them. The stacked system has
    a rank-1 Jacobian (two equal rows) and is SINGULAR. Expected counts from the exact recurrence
    in rationals; convergence is ||F|| = sqrt(2) |r^2 - 1| < tol."""
    from fractions import Fraction
    P = prob(_two_sphere_block_scene())
    u = np.array([0.48, -0.6, 0.64])
    tol = 1e-6
    for r0 in (0.9, 0.5, 0.1, 3.0):
        r, k = Fraction(r0), 0
        while not (math.sqrt(2) * abs(float(r * r - 1)) < tol):
            for _ in range(2):
                r = (r + 1 / r) / 2
            k += 1
        qo, st, it, rs = P.project((r0 * u)[None], tol=tol, max_iter=50, mode="cyclic")
        assert st[0] == CONV and it[0] == k, (r0, st[0], it[0], k)
        np.testing.assert_allclose(qo[0], float(r) * u, rtol=1e-13)
        qs, ss, _, _ = P.project((r0 * u)[None], tol=tol, max_iter=50)
        assert ss[0] == SING


def test_cyclic_split_rows_converge_to_analytic_ik(oracle_mod):
    """Planar 2R arm with the tip's x and y rows as two separate blocks: the cyclic iteration ends
    on the analytic inverse-kinematics solution (one of the two elbow branches)."""
    import dataclasses
    l1, l2, tgt = 0.7, 0.5, (0.55, 0.62)
    sc = S.planar2_scene(l1, l2, tgt)
    bx = dataclasses.replace(sc.blocks[0], mask=0x1)
    by = dataclasses.replace(sc.blocks[0], mask=0x2)
    P = prob(dataclasses.replace(sc, blocks=[bx, by]))
    x, y = tgt
    c2 = (x * x + y * y - l1 * l1 - l2 * l2) / (2 * l1 * l2)
    sols = []
    for sgn in (1, -1):
        q2 = sgn * math.acos(c2)
        q1 = math.atan2(y, x) - math.atan2(l2 * math.sin(q2), l1 + l2 * math.cos(q2))
        sols.append(np.array([q1, q2]))
    starts = np.array([[0.3, 0.9], [1.2, -0.8], [0.5, 1.5], [0.0, -1.2]])
    qo, st, it, rs = P.project(starts, tol=1e-12, max_iter=500, mode="cyclic")
    assert (st == CONV).all()
    for q in qo:
        wrapped = [np.abs((q - s + np.pi) % (2 * np.pi) - np.pi).max() for s in sols]
        assert min(wrapped) < 1e-9, (q, sols)


def test_cyclic_divergence_leaves_the_iterate(oracle_mod):
    """The MaxDistance test applies to the whole iteration: from r = 0.1 the first cycle moves the
    point by about 2.9 > 1, so the projection stops as DIVERGED with the input untouched."""
    P = prob(_two_sphere_block_scene())
    q0 = np.array([[0.1, 0.0, 0.0]])
    qo, st, it, rs = P.project(q0, tol=1e-6, max_iter=50, max_step=1.0, mode="cyclic")
    assert st[0] == DIV and it[0] == 0
    np.testing.assert_array_equal(qo, q0)


def test_cyclic_with_one_block_is_the_stacked_iteration(oracle_mod):
    """With a single constraint block a cycle is one step of the stacked system."""
    P = prob(S.sphere_scene(0))
    q, _ = S.sphere_workload(0, n_seg=16)
    a = P.project(q, tol=1e-6, max_iter=50)
    b = P.project(q, tol=1e-6, max_iter=50, mode="cyclic")
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# ---------------------------------------------------------------- interpolation (Alg. 2, interpolation step)
def test_interpolate_interior_points_are_equally_spaced_chord_points(oracle_mod):
    """Geodesic g with L_g points: the points lie on the chord a -> b, strictly inside it, spaced
    (b - a) / (L_g + 1) apart from a on, and the last one sits (b - a) / (L_g + 1) before b; an empty
    geodesic contributes nothing. Checked against exact rationals for a small integer case."""
    from fractions import Fraction
    import oracle
    rng = np.random.default_rng(4)
    e = rng.standard_normal((4, 2, 5))
    offs = np.array([0, 3, 3, 10, 11], np.int32)  # lengths 3, 0, 7, 1
    out = oracle.interpolate_interior(e, offs)
    assert out.shape == (11, 5)
    for g in range(4):
        L = offs[g + 1] - offs[g]
        pts = out[offs[g]:offs[g + 1]]
        a, b = e[g, 0], e[g, 1]
        if L == 0:
            continue
        step = (b - a) / (L + 1)
        np.testing.assert_allclose(pts[0] - a, step, atol=1e-14)
        np.testing.assert_allclose(b - pts[-1], step, atol=1e-14)
        np.testing.assert_allclose(np.diff(pts, axis=0), np.broadcast_to(step, (L - 1, 5)), atol=1e-14)
    # integers: a = (0, 3), b = (4, -1), 3 points at t = 1/4, 2/4, 3/4
    e2 = np.array([[[0.0, 3.0], [4.0, -1.0]]])
    got = oracle.interpolate_interior(e2, np.array([0, 3]))
    want = [[float(Fraction(4 * k, 4)), float(3 - Fraction(4 * k, 4))] for k in (1, 2, 3)]
    np.testing.assert_array_equal(got, want)


# ---------------------------------------------------------------- path record used by the parity band
def test_path_record_tolerance_distance_follows_heron(oracle_mod):
    """On the sphere the convergence tests see |r_k^2 - 1| of the Heron radii: the record's column 3
    is the smallest max(t / tol, tol / t) over them; no pose block, so column 2 stays 0; the longest
    step is the longest radial step and the smallest singular value 2 min r_k over the steps taken."""
    P = prob(S.sphere_scene(0))
    u = np.array([0.0, 0.6, 0.8])
    for r0 in (0.5, 0.9, 2.0):
        r, tests, steps, radii = r0, [], [], []
        while True:
            tests.append(abs(r * r - 1.0))
            if tests[-1] < 1e-6:
                break
            rn = 0.5 * (r + 1.0 / r)
            steps.append(abs(rn - r))
            radii.append(r)
            r = rn
        want = min(max(t / 1e-6, 1e-6 / t) for t in tests)
        _, st, it, _, pi = P.project((r0 * u)[None], tol=1e-6, max_iter=50, path_info=True)
        assert st[0] == CONV
        np.testing.assert_allclose(pi[0, 3], want, rtol=1e-7)  # r^2 - 1 cancels near r = 1
        assert pi[0, 2] == 0.0
        np.testing.assert_allclose(pi[0, 1], max(steps), rtol=1e-12)
        np.testing.assert_allclose(pi[0, 0], 2 * min(radii), rtol=1e-9)  # sigma(J) = 2 ||q|| at each step


def test_path_record_rotation_angle_of_a_pose_error(oracle_mod):
    """One revolute joint about z carrying a frame with a full pose block whose target rotation is
    theta_ref about z: the rotation error at q0 is |q0 - theta_ref| (wrapped to [0, pi]) and the
    iteration only reduces it, so the record's column 2 is the initial angle."""
    I = np.eye(3)
    th = 0.4
    Rr = Rotation.from_rotvec([0, 0, th]).as_matrix()
    joints = [S.Joint(-1, S.JOINT_REV, 2, I, np.zeros(3))] + \
        [S.Joint(k, S.JOINT_REV, 2, I, np.array([0.5, 0, 0])) for k in range(5)]
    blk = S.Block(S.BLK_POSE, fa=0, mask=0x3F, R=Rr, p=np.zeros(3))
    sc = S.Scene(family=S.FAMILY_PLANAR2, d=6, m=6, joints=joints, masses=np.ones(6), coms=np.zeros((6, 3)),
                 frames=[S.Frame(0, I, np.zeros(3))], blocks=[blk], spheres=np.zeros((0, 5)),
                 obstacles=np.zeros((0, 4)))
    P = prob(sc)
    for q0, ang in ((3.2, 2.8), (-2.3, 2.7), (1.0, 0.6)):
        q = np.array([[q0, 0.7, 0.1, 0.2, 0.3, 0.4]])
        _, st, _, _, pi = P.project(q, tol=1e-9, max_iter=50, lam=1e-3, path_info=True)
        np.testing.assert_allclose(pi[0, 2], ang, rtol=1e-12)


# ---------------------------------------------------------------- condition estimate of the FP64 switch
def test_kappa_est_linear_closed_forms(oracle_mod):
    """F = A q - b has J = A. Orthogonal rows of norms 1, 3, 10: J J^T = diag(1, 9, 100), so the
    Cholesky diagonal is (1, 3, 10) and kappa_est = 100 = kappa_2. General A: kappa_est equals the
    ratio from numpy's Cholesky of A A^T, and never exceeds kappa_2 (numpy's singular values)."""
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((6, 6)))
    A = np.diag([1.0, 3.0, 10.0]) @ Q[:3]
    P = prob(S.linear_scene(A, np.zeros(3)))
    ke, k2 = P.kappa_est(np.zeros((1, 6)))
    np.testing.assert_allclose([ke[0], k2[0]], [100.0, 100.0], rtol=1e-12)
    rng = np.random.default_rng(9)
    for m, d in ((2, 5), (4, 8), (6, 8)):
        A = rng.standard_normal((m, d)) * rng.uniform(0.1, 10.0, (m, 1))
        P = prob(S.linear_scene(A, np.zeros(m)))
        ke, k2 = P.kappa_est(rng.standard_normal((3, d)))
        L = np.linalg.cholesky(A @ A.T)
        dg = np.diag(L)
        np.testing.assert_allclose(ke, (dg.max() / dg.min()) ** 2, rtol=1e-10)
        sv = np.linalg.svd(A, compute_uv=False)
        np.testing.assert_allclose(k2, (sv.max() / sv.min()) ** 2, rtol=1e-9)
        assert (ke <= k2 * (1 + 1e-12)).all()
    # a rank-deficient Gram: a pivot is not positive
    A = np.array([[1.0, 2.0, 0.0], [2.0, 4.0, 0.0]])
    ke, _ = prob(S.linear_scene(A, np.zeros(2))).kappa_est(np.zeros((1, 3)))
    assert ke[0] == np.inf or ke[0] > 1e28


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_kappa_est_is_a_lower_bound_of_kappa2(oracle_mod, name):
    """(max L_ii / min L_ii)^2 <= kappa_2(J J^T) for any SPD Gram (the diagonal of L is bounded by the
    extreme singular values), on the robots' own Jacobians."""
    from parity import config_inputs
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=4)
    ke, k2 = P.kappa_est(q)
    fin = np.isfinite(ke)
    assert fin.mean() > 0.99
    assert (ke[fin] <= k2[fin] * (1 + 1e-9)).all()


# ---------------------------------------------------------------- exact derivative of the projection map
def test_vjp_exact_sphere_closed_form_off_manifold(oracle_mod):
    """The converged sphere projection is q0 / ||q0||, whose derivative (I - q^ q^T) / ||q0|| holds at
    every input, near the origin and far outside the sphere alike."""
    P = prob(S.sphere_scene(0))
    rng = np.random.default_rng(21)
    u = rng.standard_normal((6, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    q0 = u * np.array([0.05, 0.3, 0.9, 1.1, 2.5, 7.0])[:, None]
    g = rng.standard_normal((6, 3))
    gi, st = P.vjp_exact(q0, g)
    assert (st == CONV).all()
    r = np.linalg.norm(q0, axis=1, keepdims=True)
    want = (g - u * np.sum(u * g, axis=1, keepdims=True)) / r
    np.testing.assert_allclose(gi, want, atol=1e-10 * np.abs(want).max())


def test_vjp_exact_linear_steps_closed_form(oracle_mod):
    """F = A q - b: one min-norm step lands on the manifold from anywhere, so the map's derivative is
    I - A^+ A at every input. With damping lambda and step scale alpha every step is the same linear
    map q -> q - M (q - q*), M = alpha (A^T A + lambda I)^-1 A^T A, so after the oracle's K steps and
    the one past convergence the derivative is (I - M)^(K+1)."""
    rng = np.random.default_rng(22)
    A = rng.standard_normal((3, 6))
    b = rng.standard_normal(3)
    P = prob(S.linear_scene(A, b))
    q0 = 3.0 * rng.standard_normal((4, 6))
    g = rng.standard_normal((4, 6))
    gi, st = P.vjp_exact(q0, g)
    Pr = np.eye(6) - np.linalg.pinv(A) @ A
    np.testing.assert_allclose(gi, g @ Pr.T, atol=1e-11)
    lam, alpha = 0.3, 0.8
    gi, st = P.vjp_exact(q0, g, tol=1e-10, max_iter=400, alpha=alpha, lam=lam)
    _, st2, it, _ = P.project(q0, tol=1e-10, max_iter=400, alpha=alpha, lam=lam)
    assert (st == CONV).all() and (st2 == CONV).all()
    M = alpha * np.linalg.solve(A.T @ A + lam * np.eye(6), A.T @ A)
    for k in range(4):
        D = np.linalg.matrix_power(np.eye(6) - M, int(it[k]) + 1)  # dq_(K+1) / dq_0
        np.testing.assert_allclose(gi[k], D.T @ g[k], atol=1e-11)


@pytest.mark.parametrize("name", ["c1", "c4"])
def test_vjp_exact_matches_fd_of_the_projection_off_manifold(oracle_mod, name):
    """At the raw (off-manifold) inputs of the arm and humanoid batches: central differences (h = 1e-6)
    of the oracle's projection run to ||F|| < 1e-13 (the converged map) against the forward-mode
    derivative, relative error in ||g_in||."""
    from parity import config_inputs
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=1)
    q = q[:6]
    _, st0, _, _, pi = P.project(q, tol=1e-13, max_iter=100, path_info=True)
    keep = (st0 == CONV) & (pi[:, 0] > 1e-2) & (pi[:, 1] < 1.0)  # well-conditioned paths, FD is meaningful
    q = q[keep]
    assert len(q) >= 3
    rng = np.random.default_rng(23)
    g = rng.standard_normal(q.shape)
    gi, st = P.vjp_exact(q, g)
    h, d = 1e-6, sc.d
    qp = np.repeat(q, d, axis=0) + h * np.tile(np.eye(d), (len(q), 1))
    qm = np.repeat(q, d, axis=0) - h * np.tile(np.eye(d), (len(q), 1))
    pp = P.project(qp, tol=1e-13, max_iter=100)[0]
    pm = P.project(qm, tol=1e-13, max_iter=100)[0]
    dP = ((pp - pm) / (2 * h)).reshape(len(q), d, d)  # [n, i (input), :] = dP / dq_i
    g_fd = np.einsum("nij,nj->ni", dP, g)
    rel = np.linalg.norm(gi - g_fd, axis=1) / np.linalg.norm(g_fd, axis=1)
    assert rel.max() < 1e-5, rel
    # off the manifold the exact derivative is not the tangent projector at the output
    go, _ = P.vjp(P.project(q, tol=1e-13, max_iter=100)[0], g)
    assert (np.linalg.norm(go - g_fd, axis=1) / np.linalg.norm(g_fd, axis=1)).max() > 1e-4


def test_vjp_exact_on_the_manifold_is_the_tangent_projector(oracle_mod):
    """From an input already on the manifold the converged map's derivative is I - J^+ J there."""
    from parity import config_inputs
    sc, P, q, offs, tol, mi = config_inputs("c3", small=True, max_geo=1)
    q = P.project(q[:4], tol=1e-14, max_iter=100)[0]
    g = np.random.default_rng(24).standard_normal(q.shape)
    gi, st = P.vjp_exact(q, g, tol=1e-13)
    go, _ = P.vjp(q, g)
    assert (st == CONV).all()
    np.testing.assert_allclose(gi, go, atol=1e-8 * np.abs(go).max())
