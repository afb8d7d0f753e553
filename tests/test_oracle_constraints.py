"""Pins of the oracle's paper-only constraint rows (no GPU): finite TSR bounds (Sec. III, B^w),
the closed-linkage rod lengths and the CoM-within-support-polygon rows of the Digit constraint figure,
and the pseudo-inverse step the oracle takes where those rows make the Jacobian's rank vary.

Each test checks the oracle against something other than itself: closed forms of one Newton step
on robots whose kinematics are linear (prismatic chains), brute force over a densely sampled polygon
boundary, numpy's pseudo-inverse of the oracle's own Jacobian, and invariants of converged Digit
configurations computed from link and frame poses alone (no residual code)."""
import math

import numpy as np
import pytest

from paper_2604_13323_amd import scenes as S

CONV, MAXIT, SING, DIV, NONF = range(5)
PRI, REV = S.JOINT_PRI, S.JOINT_REV
I3 = np.eye(3)


def prob(scene):
    import oracle
    return oracle.Problem(scene.to_blob())


def chain(axes, parent0=-1, index0=0, jtype=S.JOINT_PRI):
    """Serial chain of joints about / along the given axes, all origins at zero."""
    return [S.Joint(parent0 if i == 0 else index0 + i - 1, jtype, a, I3, np.zeros(3)) for i, a in enumerate(axes)]


def point_hull_scene(poly):
    """A point mass on an x-y prismatic chain: its CoM xy is (q0, q1)."""
    joints = chain([0, 1])
    return S.Scene(family=99, d=2, m=2, joints=joints, masses=np.array([0.0, 1.0]), coms=np.zeros((2, 3)),
                   frames=[S.Frame(1, I3, np.zeros(3))], blocks=[S.hull_block(poly)],
                   spheres=np.zeros((0, 5)), obstacles=np.zeros((0, 4)))


def two_points_dist_scene(L=0.0, qref=None):
    """Two points, each on its own x-y-z prismatic chain (6 DoF), a rod of length L between them."""
    joints = chain([0, 1, 2]) + chain([0, 1, 2], parent0=-1, index0=3)
    return S.Scene(family=99, d=6, m=1, joints=joints, masses=np.zeros(6), coms=np.zeros((6, 3)),
                   frames=[S.Frame(2, I3, np.zeros(3)), S.Frame(5, I3, np.zeros(3))],
                   blocks=[S.dist_block(0, 1, L, from_qref=qref is not None)], spheres=np.zeros((0, 5)),
                   obstacles=np.zeros((0, 4)), qref=qref)


def point_box_scene(lo, hi, p_ref):
    """A point on an x-y-z prismatic chain with a TSR on its translation rows, bounds [lo, hi]."""
    lo6 = np.concatenate([lo, [-np.inf] * 3])
    hi6 = np.concatenate([hi, [np.inf] * 3])
    return S.Scene(family=99, d=3, m=3, joints=chain([0, 1, 2]), masses=np.zeros(3), coms=np.zeros((3, 3)),
                   frames=[S.Frame(2, I3, np.zeros(3))], blocks=[S.bounded_pose_block(0, lo6, hi6, p=p_ref, mask=0x7)],
                   spheres=np.zeros((0, 5)), obstacles=np.zeros((0, 4)))


def yaw_joint_scene(lo, hi, mask=0x20):
    """One revolute joint about z with a TSR on the rotation rows selected by mask."""
    lo6 = np.array([-np.inf] * 3 + list(lo))
    hi6 = np.array([np.inf] * 3 + list(hi))
    m = bin(mask).count("1")
    return S.Scene(family=99, d=1, m=m, joints=chain([2], jtype=REV), masses=np.zeros(1), coms=np.zeros((1, 3)),
                   frames=[S.Frame(0, I3, np.zeros(3))], blocks=[S.bounded_pose_block(0, lo6, hi6, mask=mask)],
                   spheres=np.zeros((0, 5)), obstacles=np.zeros((0, 4)))


def brute_nearest_on_polygon(poly, x, n=40001):
    """Nearest point of the polygon's boundary to x by dense sampling (each edge n points)."""
    best, bp = np.inf, None
    t = np.linspace(0.0, 1.0, n)[:, None]
    for i in range(len(poly)):
        a, b = poly[i], poly[(i + 1) % len(poly)]
        pts = a + t * (b - a)
        d2 = np.sum((pts - x) ** 2, axis=1)
        k = int(np.argmin(d2))
        if d2[k] < best:
            best, bp = d2[k], pts[k]
    return bp


def inside_polygon(poly, x):
    def cross(u, v):
        return u[0] * v[1] - u[1] * v[0]
    return all(cross(poly[(i + 1) % len(poly)] - poly[i], x - poly[i]) >= 0 for i in range(len(poly)))


PENTAGON = np.array([[0.0, 0.0], [1.0, -0.2], [1.4, 0.6], [0.7, 1.3], [-0.2, 0.8]])


# ---------------------------------------------------------------- CoM within the support polygon
def test_polygon_rows_zero_inside_and_point_minus_nearest_outside(oracle_mod):
    P = prob(point_hull_scene(PENTAGON))
    rng = np.random.default_rng(11)
    X = rng.uniform(-1.0, 2.5, (300, 2))
    F = P.residual(X)
    for x, f in zip(X, F):
        if inside_polygon(PENTAGON, x):
            assert np.all(f == 0.0)
        else:
            np.testing.assert_allclose(f, x - brute_nearest_on_polygon(PENTAGON, x), atol=3e-5)


def test_unit_square_projection_one_step_closed_forms(oracle_mod):
    """Projecting a point mass onto the unit square: edge regions land on the foot of the
    perpendicular, vertex regions on the vertex, both in one step; inside points take none."""
    sq = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    P = prob(point_hull_scene(sq))
    cases = [((2.0, 0.5), (1.0, 0.5), 1), ((0.5, -3.0), (0.5, 0.0), 1), ((2.0, 2.0), (1.0, 1.0), 1),
             ((-1.0, -0.25), (0.0, 0.0), 1), ((-0.5, 0.7), (0.0, 0.7), 1), ((0.3, 0.4), (0.3, 0.4), 0)]
    X = np.array([c[0] for c in cases])
    qo, st, it, rs = P.project(X, tol=1e-9, max_iter=10)
    assert np.all(st == CONV)
    for (x, want, k), q, n in zip(cases, qo, it):
        assert n == k, (x, n)
        np.testing.assert_allclose(q, want, atol=1e-15)


def test_polygon_projection_is_the_nearest_point(oracle_mod):
    """From random points, the converged point is the Euclidean projection onto the polygon."""
    P = prob(point_hull_scene(PENTAGON))
    X = np.random.default_rng(12).uniform(-1.5, 3.0, (200, 2))
    qo, st, it, rs = P.project(X, tol=1e-12, max_iter=10)
    assert np.all(st == CONV) and np.all(it <= 1)
    for x, q in zip(X, qo):
        want = x if inside_polygon(PENTAGON, x) else brute_nearest_on_polygon(PENTAGON, x)
        np.testing.assert_allclose(q, want, atol=3e-5)


def test_polygon_jacobian_rank_and_path_sigma(oracle_mod):
    """Edge region: J = n n^T (rank 1), the path record's sigma_min is its nonzero singular value 1;
    vertex region: J = I; inside: J = 0."""
    sq = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    P = prob(point_hull_scene(sq))
    J = P.jacobian(np.array([[2.0, 0.5], [2.0, 2.0], [0.5, 0.5]]))
    np.testing.assert_allclose(J[0], [[1.0, 0.0], [0.0, 0.0]], atol=1e-15)
    np.testing.assert_allclose(J[1], np.eye(2), atol=1e-15)
    np.testing.assert_allclose(J[2], np.zeros((2, 2)), atol=0)
    _, st, it, rs, pi = P.project(np.array([[2.0, 0.5], [2.0, 2.0]]), tol=1e-9, max_iter=5, path_info=True)
    np.testing.assert_allclose(pi[:, 0], [1.0, 1.0], rtol=1e-12)


def test_polygon_tangent_vjp_edge_region_and_inside(oracle_mod):
    """Tangent projector just outside an edge: I - n n^T (the rows' row space is n); inside: I."""
    sq = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    P = prob(point_hull_scene(sq))
    g = np.array([[0.3, -0.7], [0.3, -0.7]])
    gi, _ = P.vjp(np.array([[1.0 + 1e-9, 0.4], [0.5, 0.5]]), g)
    np.testing.assert_allclose(gi[0], [0.0, -0.7], atol=1e-15)
    np.testing.assert_allclose(gi[1], g[1], atol=0)


def test_bad_polygon_is_rejected(oracle_mod):
    import oracle
    cw = PENTAGON[::-1].copy()
    with pytest.raises(ValueError):
        oracle.Problem(point_hull_scene(cw).to_blob())
    notconvex = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 0.2], [1.0, 1.0], [0.0, 1.0]])
    with pytest.raises(ValueError):
        oracle.Problem(point_hull_scene(notconvex).to_blob())


# ---------------------------------------------------------------- closed linkage
def test_rod_one_step_restores_length_symmetrically(oracle_mod):
    """F = ||p_b - p_a|| - L is linear along the rod: the min-norm step moves both ends by F/2 along
    it, so one step gives the length exactly, keeps the midpoint and the direction."""
    L = 0.7
    P = prob(two_points_dist_scene(L))
    rng = np.random.default_rng(13)
    Q = rng.normal(0.0, 1.0, (50, 6))
    qo, st, it, rs = P.project(Q, tol=1e-9, max_iter=5)
    assert np.all(st == CONV) and np.all(it == 1)
    for q, o in zip(Q, qo):
        a, b, a2, b2 = q[:3], q[3:], o[:3], o[3:]
        assert abs(np.linalg.norm(b2 - a2) - L) < 1e-14
        np.testing.assert_allclose(a2 + b2, a + b, atol=1e-14)
        u, u2 = (b - a) / np.linalg.norm(b - a), (b2 - a2) / L
        np.testing.assert_allclose(u2, u, atol=1e-14)
    F = P.residual(Q)
    np.testing.assert_allclose(F[:, 0], np.linalg.norm(Q[:, 3:] - Q[:, :3], axis=1) - L, rtol=1e-14)


def test_rod_length_taken_at_the_reference_configuration(oracle_mod):
    qref = np.array([0.1, 0.2, 0.3, 1.1, -0.4, 0.9])
    P = prob(two_points_dist_scene(qref=qref))
    L = np.linalg.norm(qref[3:] - qref[:3])
    assert abs(P.residual(qref[None])[0, 0]) < 1e-15
    q = qref + 0.1
    q[5] += 0.3
    np.testing.assert_allclose(P.residual(q[None])[0, 0], np.linalg.norm(q[3:] - q[:3]) - L, rtol=1e-14)


# ---------------------------------------------------------------- finite TSR bounds
def test_translation_box_one_step_is_the_clamp(oracle_mod):
    lo, hi, pr = np.array([-0.2, -0.1, 0.0]), np.array([0.3, 0.1, 0.5]), np.array([1.0, 2.0, 3.0])
    P = prob(point_box_scene(lo, hi, pr))
    rng = np.random.default_rng(14)
    Q = pr + np.concatenate([rng.uniform(-1.0, 1.0, (100, 3)), rng.uniform(lo, hi, (20, 3))])
    qo, st, it, rs = P.project(Q, tol=1e-12, max_iter=5)
    want = pr + np.clip(Q - pr, lo, hi)
    assert np.all(st == CONV)
    np.testing.assert_allclose(qo, want, atol=1e-15)
    inside = np.all((Q - pr >= lo) & (Q - pr <= hi), axis=1)
    assert np.all(it[inside] == 0) and np.all(it[~inside] == 1) and inside.any()
    F = P.residual(Q)
    np.testing.assert_allclose(F, (Q - pr) - np.clip(Q - pr, lo, hi), atol=1e-15)


def test_rotation_bound_one_step(oracle_mod):
    """log(R_z(q)) = (0, 0, q) for |q| < pi: the yaw row is linear in q, so one step clamps q to its
    interval."""
    P = prob(yaw_joint_scene([-np.inf, -np.inf, -0.3], [np.inf, np.inf, 0.5], mask=0x20))
    Q = np.array([[1.2], [-1.0], [0.1], [0.5]])
    qo, st, it, rs = P.project(Q, tol=1e-12, max_iter=5)
    assert np.all(st == CONV)
    np.testing.assert_allclose(qo[:, 0], [0.5, -0.3, 0.1, 0.5], atol=1e-15)
    assert list(it) == [1, 1, 0, 0]
    np.testing.assert_allclose(P.residual(Q)[:, 0], [0.7, -0.7, 0.0, 0.0], atol=1e-15)


def test_free_component_contributes_nothing(oracle_mod):
    """A component with infinite bounds is a zero row with a zero Jacobian row; the others clamp."""
    lo, hi, pr = np.array([-np.inf, -0.1, 0.0]), np.array([np.inf, 0.1, 0.5]), np.zeros(3)
    P = prob(point_box_scene(lo, hi, pr))
    Q = np.random.default_rng(15).uniform(-2.0, 2.0, (40, 3))
    assert np.all(P.residual(Q)[:, 0] == 0.0) and np.all(P.jacobian(Q)[:, 0, :] == 0.0)
    qo, st, it, rs = P.project(Q, tol=1e-12, max_iter=5)
    np.testing.assert_allclose(qo, np.clip(Q, lo, hi), atol=1e-15)


def test_inverted_bounds_are_rejected(oracle_mod):
    import oracle
    with pytest.raises(ValueError):
        oracle.Problem(point_box_scene(np.array([0.1, 0, 0]), np.array([0.0, 1, 1]), np.zeros(3)).to_blob())


# ---------------------------------------------------------------- the pseudo-inverse step
@pytest.mark.parametrize("name", ["c5", "c6"])
def test_step_is_numpy_pinv_of_the_jacobian(oracle_mod, name):
    """One Newton step from the raw batch equals q - pinv(J) F with numpy's SVD-based pseudo-inverse
    of the oracle's own Jacobian and residual (rank cut 1e-10 sigma_max)."""
    import oracle
    cfg = S.make_config(name, small=True)
    sc = cfg["scene"]
    P = prob(sc)
    if "q" in cfg:
        q = cfg["q"][:64]
    else:
        e = cfg["endpoints"][:4].reshape(-1, sc.d)
        q = oracle.interpolate_interior(P.project(e, tol=1e-10, max_iter=100)[0].reshape(-1, 2, sc.d),
                                        np.array([0, 32, 64, 96, 128], np.int32))[:64]
    F = P.residual(q)
    J = P.jacobian(q)
    q1, st, it, rs = P.project(q, tol=1e-300, max_iter=1)
    moved = it == 1
    assert moved.sum() >= 32
    rank_def = 0
    for i in np.nonzero(moved)[0]:
        want = q[i] - np.linalg.pinv(J[i], rcond=1e-10) @ F[i]
        np.testing.assert_allclose(q1[i], want, atol=1e-12 * max(1.0, np.abs(q[i]).max()))
        rank_def += int(np.linalg.matrix_rank(J[i], tol=1e-10 * np.linalg.norm(J[i], 2)) < sc.m)
    assert rank_def > 0  # the batch has configurations with inactive or rank-deficient rows


def test_vjp_exact_refuses_piecewise_rows(oracle_mod):
    P = prob(point_hull_scene(PENTAGON))
    with pytest.raises(NotImplementedError):
        P.vjp_exact(np.array([[2.0, 0.5]]), np.ones((1, 2)))


# ---------------------------------------------------------------- the Digit constraint set
def _rot_angle(R):
    """Rotation angle from ||R - I||_F = 2 sqrt(2) sin(theta / 2) (accurate near zero)."""
    return 2.0 * math.asin(min(1.0, np.linalg.norm(R - np.eye(3)) / (2.0 * math.sqrt(2.0))))


def test_digit_converged_configurations_satisfy_every_constraint(oracle_mod):
    """From link and frame poses alone: feet at their target poses, hands at their relative pose
    at q_ref, both rods at their q_ref lengths, and the CoM xy inside the support polygon or within
    tol of it (polygon distance by brute force)."""
    import oracle
    cfg = S.make_config("c5", small=True)
    sc = cfg["scene"]
    P = prob(sc)
    e = cfg["endpoints"][:8].reshape(-1, sc.d)
    tol = 1e-9
    qo, st, it, rs = P.project(e, tol=tol, max_iter=100)
    assert (st == CONV).mean() > 0.9
    fr_ref = P.frame_poses(sc.qref)
    rel_ref = np.linalg.inv(_T(fr_ref[2])) @ _T(fr_ref[3])
    L_ref = [np.linalg.norm(fr_ref[5, 9:] - fr_ref[4, 9:]), np.linalg.norm(fr_ref[7, 9:] - fr_ref[6, 9:])]
    poly = sc.blocks[3].ext[:2 * sc.blocks[3].aux].reshape(-1, 2)
    M = sc.masses.sum()
    for q in qo[st == CONV]:
        fr = P.frame_poses(q)
        for f, b in ((0, sc.blocks[0]), (1, sc.blocks[1])):
            T = _T(fr[f])
            assert np.linalg.norm(T[:3, 3] - b.p) < tol and _rot_angle(b.R.T @ T[:3, :3]) < tol
        rel = np.linalg.inv(_T(fr[2])) @ _T(fr[3])
        assert np.linalg.norm(rel[:3, 3] - rel_ref[:3, 3]) < tol
        assert _rot_angle(rel_ref[:3, :3].T @ rel[:3, :3]) < tol
        assert abs(np.linalg.norm(fr[5, 9:] - fr[4, 9:]) - L_ref[0]) < tol
        assert abs(np.linalg.norm(fr[7, 9:] - fr[6, 9:]) - L_ref[1]) < tol
        lf = P.link_frames(q)
        c = np.zeros(2)
        for l in range(sc.d):
            R, p = lf[l, :9].reshape(3, 3), lf[l, 9:]
            c += sc.masses[l] * (R @ sc.coms[l] + p)[:2]
        c /= M
        if not inside_polygon(poly, c):  # then within tol of some edge's line, between its ends
            dist = []
            for i in range(len(poly)):
                a, b = poly[i], poly[(i + 1) % len(poly)]
                e = (b - a) / np.linalg.norm(b - a)
                t = float(np.dot(c - a, e))
                if -tol <= t <= np.linalg.norm(b - a) + tol:
                    dist.append(abs(e[0] * (c - a)[1] - e[1] * (c - a)[0]))
            assert min(dist) < tol


def _T(row):
    T = np.eye(4)
    T[:3, :3] = row[:9].reshape(3, 3)
    T[:3, 3] = row[9:]
    return T


def test_digit_scene_polygon_is_the_hull_of_the_soles(oracle_mod):
    """The support polygon stored in the scene contains every sole-patch corner and each of its
    vertices is one of them."""
    sc = S.digit36_scene(5)
    poly = sc.blocks[3].ext[:2 * sc.blocks[3].aux].reshape(-1, 2)
    corners = []
    for b, yaw in ((sc.blocks[0], S.DIGIT_TOE_OUT), (sc.blocks[1], -S.DIGIT_TOE_OUT)):
        for x in S.DIGIT_SOLE_X:
            for y in S.DIGIT_SOLE_Y:
                c = np.array([x * math.cos(yaw) - y * math.sin(yaw), x * math.sin(yaw) + y * math.cos(yaw)])
                corners.append(c + b.p[:2])
    corners = np.array(corners)
    for c in corners:
        assert inside_polygon(poly, c) or np.min(np.linalg.norm(poly - c, axis=1)) < 1e-12
    for v in poly:
        assert np.min(np.linalg.norm(corners - v, axis=1)) < 1e-12
