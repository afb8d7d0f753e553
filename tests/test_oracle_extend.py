"""Pins of the oracle's ConstrainedExtend (Alg. 2; Sec. IV-A and IV-B) to closed forms.

On the unit sphere (F = q.q - 1) the projection of a point p is p / ||p|| after the Heron
recurrence r <- (r + 1/r) / 2 on r = ||p||, and the normalised chord point between two unit
vectors at angles a, b of one plane lies at the angle atan2(t sin(b-a), 1 - t + t cos(b-a)) from a;
the midpoint of two unit vectors, normalised, lies at the mean angle. On an affine constraint
(F = A q - b) points already on the manifold take no step and every chord between two of them
stays on it, so all gaps of a chain are exact fractions of its length. The worked cases below are
chosen with wide margins on every threshold the method tests."""
import math

import numpy as np
import pytest

import oracle
from oracle import extend as OX
from paper_2604_13323_amd import scenes as S


def sphere_problem(obstacles=((10.0, 10.0, 10.0, 0.1),)):
    sc = S.Scene(family=S.FAMILY_SPHERE, d=3, m=1, joints=[], masses=np.zeros(0), coms=np.zeros((0, 3)),
                 blocks=[S.Block(S.BLK_SPHERE)], spheres=np.array([[-1, 0, 0, 0, 0.0]]),
                 obstacles=np.asarray(obstacles, np.float64).reshape(-1, 4), name="sphere3")
    return oracle.Problem(sc.to_blob())


def heron_steps(r0, tol):
    r, k = r0, 0
    while abs(r * r - 1.0) >= tol:
        r = 0.5 * (r + 1.0 / r)
        k += 1
    return k


def chord_angle(t, phi):
    return math.atan2(t * math.sin(phi), 1.0 - t + t * math.cos(phi))


S0 = np.array([1.0, 0.0, 0.0])
T0 = np.array([0.0, 1.0, 0.0])
V0 = (T0 - S0) / np.linalg.norm(T0 - S0)


def angle_of(q):
    return math.atan2(q[1], q[0])


def test_sphere_steer_and_projection_of_the_selected_particle():
    P = sphere_problem()
    eps = np.zeros(4)
    code, best, qp, chain = OX.extend_one(P, S0, T0, eps, r=0.5, delta=0.2, tol=1e-10, max_iter=50)
    steer = S0 + 0.5 * V0  # min(||t - s||, r) = 0.5 along v
    np.testing.assert_allclose(qp, steer / np.linalg.norm(steer), atol=1e-12)
    assert best == 0  # identical particles: the lowest index
    assert code == OX.OK


def test_sphere_earliest_particle_is_the_one_with_fewest_heron_steps():
    P = sphere_problem()
    eps = np.array([0.6, 0.3, 0.1, 0.02, 0.45, 0.05]) - 0.5  # Heron steps 4, 4, 3, 2, 4, 3 at tol 1e-8
    tol = 1e-8
    norms = [np.linalg.norm(S0 + (0.5 + e) * V0) for e in eps]
    steps = [heron_steps(r0, tol) for r0 in norms]
    want = int(np.argmin(steps))
    assert steps.count(min(steps)) == 1, "case must have a unique earliest particle"
    code, best, qp, _ = OX.extend_one(P, S0, T0, eps, r=0.5, delta=0.2, tol=tol, max_iter=50)
    assert best == want
    p = S0 + (0.5 + eps[want]) * V0
    np.testing.assert_allclose(qp, p / np.linalg.norm(p), atol=1e-9)


def test_sphere_earliest_ties_go_to_the_lowest_index():
    P = sphere_problem()
    # +a and the particle with the same norm on the other side of the foot point of the chord
    # (||s + a v||^2 = 1 - sqrt(2) a + a^2 is symmetric about a = 1/sqrt(2))
    a1 = 0.1
    a2 = math.sqrt(2.0) - a1
    eps = np.array([0.6 - 0.5, a2 - 0.5, a1 - 0.5])  # norms: distinct, equal, equal
    tol = 1e-8
    steps = [heron_steps(np.linalg.norm(S0 + (0.5 + e) * V0), tol) for e in eps]
    assert steps[1] == steps[2] < steps[0]
    _, best, _, _ = OX.extend_one(P, S0, T0, eps, r=0.5, delta=0.2, tol=tol, max_iter=50)
    assert best == int(np.argmin(steps))  # lowest index among the minima


def test_sphere_chain_levels_follow_the_chord_geometry():
    P = sphere_problem()
    eps = np.zeros(4)
    phi = angle_of((S0 + 0.5 * V0) / np.linalg.norm(S0 + 0.5 * V0))
    # level 0: 5 gaps between the normalised chord points k/5
    th0 = [0.0] + [chord_angle(k / 5.0, phi) for k in range(1, 5)] + [phi]
    g0 = [2 * math.sin((b - a) / 2) for a, b in zip(th0[:-1], th0[1:])]
    assert max(g0) < 0.125 - 0.01          # r / n = 0.125: passes with margin
    assert 0.06 + 0.01 < max(g0) < 0.2 - 0.05
    code, _, _, chain = OX.extend_one(P, S0, T0, eps, r=0.5, delta=0.2, tol=1e-10, max_iter=50)
    assert code == OX.OK and chain.shape[0] == 6
    np.testing.assert_allclose([angle_of(c) for c in chain], th0, atol=1e-9)
    # level 1: midpoints at the mean angles
    th1 = []
    for a, b in zip(th0[:-1], th0[1:]):
        th1 += [a, 0.5 * (a + b)]
    th1.append(th0[-1])
    g1 = [2 * math.sin((b - a) / 2) for a, b in zip(th1[:-1], th1[1:])]
    assert max(g1) < 0.06 - 0.005 and max(g1) < 0.0625
    code, _, _, chain = OX.extend_one(P, S0, T0, eps, r=0.5, delta=0.06, tol=1e-10, max_iter=50)
    assert code == OX.OK and chain.shape[0] == 11
    np.testing.assert_allclose([angle_of(c) for c in chain], th1, atol=1e-9)
    for c in chain:
        assert abs(np.linalg.norm(c) - 1.0) < 1e-9


def test_sphere_gap_and_too_far_exits():
    P = sphere_problem()
    # eps = 0.3: q_proj at angle ~0.916; 9 level-0 gaps of ~0.10 > r / n = 0.0625
    eps = np.full(8, 0.3)
    p = S0 + 0.8 * V0
    phi = angle_of(p / np.linalg.norm(p))
    assert 2 * math.sin(phi / 2) < 1.0 - 0.05       # within 2 dist: not TOO_FAR
    assert 2 * math.sin(phi / 18) > 0.0625 + 0.02    # the smallest possible level-0 gap already fails
    code, best, _, _ = OX.extend_one(P, S0, T0, eps, r=0.5, delta=0.05, tol=1e-10, max_iter=50)
    assert code == OX.GAP and best == 0
    # eps = 0.45: q_proj so far round the sphere that ||q_proj - s|| > 2 dist = 1
    eps = np.full(8, 0.45)
    p = S0 + 0.95 * V0
    phi = angle_of(p / np.linalg.norm(p))
    assert 2 * math.sin(phi / 2) > 1.0 + 0.05
    code, _, _, _ = OX.extend_one(P, S0, T0, eps, r=0.5, delta=0.05, tol=1e-10, max_iter=50)
    assert code == OX.TOO_FAR


def test_sphere_degenerate_cases():
    P = sphere_problem()
    code, best, qp, _ = OX.extend_one(P, S0, S0.copy(), np.zeros(4), r=0.5, delta=0.1, tol=1e-8, max_iter=50)
    assert code == OX.ZERO and best == -1 and qp is None
    # target opposite: the steer point with r = 1 is the origin, where every particle with eps = 0
    # sits and no step is defined
    code, best, _, _ = OX.extend_one(P, S0, -S0, np.zeros(4), r=1.0, delta=0.1, tol=1e-8, max_iter=50)
    assert code == OX.NO_PARTICLE and best == -1


def test_sphere_collision_exits():
    eps = np.zeros(4)
    steer = S0 + 0.5 * V0
    qp = steer / np.linalg.norm(steer)
    P = sphere_problem([(qp[0], qp[1], 0.0, 0.02), (10, 10, 10, 0.1)])
    code, _, _, _ = OX.extend_one(P, S0, T0, eps, r=0.5, delta=0.2, tol=1e-10, max_iter=50)
    assert code == OX.COLLISION
    # an obstacle on the second level-0 point only (its neighbours are ~0.1 away)
    phi = angle_of(qp)
    a = chord_angle(2 / 5.0, phi)
    P = sphere_problem([(math.cos(a), math.sin(a), 0.0, 0.01)])
    code, _, _, _ = OX.extend_one(P, S0, T0, eps, r=0.5, delta=0.2, tol=1e-10, max_iter=50)
    assert code == OX.INTERP_COLLISION


def linear_problem():
    A = np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0]])
    b = np.array([0.3, -0.2])
    return oracle.Problem(S.linear_scene(A, b).to_blob()), A, b


@pytest.mark.parametrize("eps0,code,npts", [(0.05, OX.OK, 11), (0.15, OX.GAP, 0), (0.45, OX.TOO_FAR, 0)])
def test_linear_manifold_chain_is_exact(eps0, code, npts):
    """Start and target both on the affine manifold {x0 = 0.3, x1 = -0.2}: the particles sit on it
    (no step), q_proj = s + (r + eps_0) e_2, and the chain gaps are (r + eps_0) / ((n + 1) 2^l)."""
    P, A, b = linear_problem()
    s = np.array([0.3, -0.2, 0.0, 0.0])
    t = np.array([0.3, -0.2, 1.0, 0.0])
    eps = np.array([eps0, 0.0, 0.01, -0.01])  # n = 4: all take 0 steps, the lowest index wins
    r, delta = 0.4, 0.05
    c, best, qp, chain = OX.extend_one(P, s, t, eps, r=r, delta=delta, tol=1e-10, max_iter=10)
    assert c == code and best == 0
    np.testing.assert_allclose(qp, s + (r + eps0) * np.array([0, 0, 1.0, 0]), atol=1e-14)
    if code == OX.OK:
        D = r + eps0
        gaps = np.linalg.norm(chain[1:] - chain[:-1], axis=1)
        np.testing.assert_allclose(gaps, D / 10.0, rtol=1e-12)  # level 1: (n + 1) 2 = 10 gaps
        assert chain.shape[0] == npts


def test_linear_off_manifold_particles_take_one_textbook_step():
    """Direction with a component across the manifold: every particle needs exactly one step, so
    the lowest index is selected and q_proj is the least-norm correction of particle 0."""
    P, A, b = linear_problem()
    s = np.array([0.3, -0.2, 0.0, 0.0])
    t = np.array([0.8, 0.1, 0.6, -0.3])
    eps = np.array([0.02, -0.03, 0.01, 0.0, 0.04])
    r = 0.5
    L = np.linalg.norm(t - s)
    v = (t - s) / L
    p0 = s + (min(L, r) + eps[0]) * v
    want = p0 - np.linalg.lstsq(A, A @ p0 - b, rcond=None)[0]
    code, best, qp, chain = OX.extend_one(P, s, t, eps, r=r, delta=0.2, tol=1e-10, max_iter=10)
    assert best == 0
    np.testing.assert_allclose(qp, want, atol=1e-13)
    D = np.linalg.norm(want - s)
    assert code == OX.OK
    gaps = np.linalg.norm(chain[1:] - chain[:-1], axis=1)
    np.testing.assert_allclose(gaps, D / (chain.shape[0] - 1), rtol=1e-10)


def test_sphere_interpolated_point_at_the_origin_fails():
    """Target opposite the start with r = 2: the steer point is the antipode itself (on the sphere, no
    step), q_proj = -s passes both first exits (||q_proj - s|| = 2 <= 2 dist = 4), and with n = 3 the
    middle interpolated point s + (q_proj - s) / 2 is the origin, where the Jacobian 2q vanishes and
    no step exists: INTERP_FAILED, with the particle selected."""
    P = sphere_problem()
    code, best, qp, chain = OX.extend_one(P, S0, -S0, np.zeros(3), r=2.0, delta=0.1, tol=1e-8, max_iter=50)
    assert code == OX.INTERP_FAILED and best == 0 and chain is None
    np.testing.assert_array_equal(qp, -S0)
