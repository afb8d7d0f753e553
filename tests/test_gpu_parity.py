"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on the same seeded
inputs. Tolerances: projected coordinates within 1e-4 (FP32 mode) and 1e-9 (FP64 mode) of the
oracle; statuses and iteration counts equal outside the band, band configurations compared as
parity.py describes; collision verdicts equal outside a 1e-5 m margin band; VJPs within 1e-3
relative (FP32) / 1e-9 (FP64)."""
import math

import numpy as np
import pytest

from parity import CONV, MAXIT, NONF, SING, band_mask, compare, config_inputs, from_dev, oracle_run, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mc():
    import paper_2604_13323_amd as M
    M.lib()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return M


def gpu_problem(mc, sc):
    return mc.Problem(sc.to_blob())


def run_gpu(mc, sc, q, tol, max_iter, dtype=torch.float32, **kw):
    G = gpu_problem(mc, sc)
    r = G.project(to_dev(q, dtype), tol=tol, max_iter=max_iter, **kw)
    torch.cuda.synchronize()
    return G, r


# ---------------------------------------------------------------- closed forms through the GPU
def test_sphere_heron_counts_and_closed_form(mc):
    from paper_2604_13323_amd import scenes as S
    sc = S.sphere_scene(0)
    rng = np.random.default_rng(7)
    radii = [0.9, 0.5, 0.1, 0.01, 3.0]
    k = [3, 4, 7, 10, 5]
    u = rng.standard_normal((5, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    q = u * np.array(radii)[:, None]
    for dt, qt in ((torch.float32, 1e-6), (torch.float64, 1e-12)):
        G, r = run_gpu(mc, sc, q, 1e-6, 50, dt)
        assert list(from_dev(r.iters).astype(int)) == k
        assert (from_dev(r.status) == CONV).all()
        np.testing.assert_allclose(from_dev(r.q).T, u, atol=1e-6 if dt == torch.float32 else 1e-6)


def test_sphere_forced_statuses(mc):
    from paper_2604_13323_amd import scenes as S
    sc = S.sphere_scene(0)
    q = np.array([[0.0, 0.0, 0.0], [np.nan, 0.0, 1.0], [0.1, 0.0, 0.0], [0.0, 0.6, 0.8]])
    for dt in (torch.float32, torch.float64):
        G, r = run_gpu(mc, sc, q, 1e-6, 1, dt)
        st = from_dev(r.status).astype(int)
        it = from_dev(r.iters).astype(int)
        assert st[0] == SING and it[0] == 0
        assert st[1] == NONF
        assert st[2] == MAXIT and it[2] == 1
        assert st[3] == CONV and it[3] == 0
        v = from_dev(r.verdict).astype(int)
        assert v[0] == 2 and v[1] == 2 and v[2] == 2


def test_linear_one_step_least_norm(mc):
    from paper_2604_13323_amd import scenes as S
    rng = np.random.default_rng(3)
    for (m, d) in [(1, 3), (2, 5), (3, 7), (4, 8), (6, 8)]:
        A = rng.standard_normal((m, d))
        b = rng.standard_normal(m)
        sc = S.linear_scene(A, b)
        q0 = rng.standard_normal((70, d))
        ref = np.stack([q0[i] - np.linalg.lstsq(A, A @ q0[i] - b, rcond=None)[0] for i in range(70)])
        for dt, qt in ((torch.float32, 2e-5), (torch.float64, 1e-11)):
            G, r = run_gpu(mc, sc, q0, 1e-5 if dt == torch.float32 else 1e-9, 10, dt)
            assert (from_dev(r.status) == CONV).all()
            np.testing.assert_allclose(from_dev(r.q).T, ref, atol=qt)


def test_planar_2r_analytic_ik(mc):
    from paper_2604_13323_amd import scenes as S
    rng = np.random.default_rng(11)
    l1, l2 = 0.7, 0.5
    for _ in range(8):
        rad, ang = rng.uniform(0.3, 1.1), rng.uniform(-math.pi, math.pi)
        x, y = rad * math.cos(ang), rad * math.sin(ang)
        sc = S.planar2_scene(l1, l2, (x, y))
        c2 = (x * x + y * y - l1 * l1 - l2 * l2) / (2 * l1 * l2)
        sols = []
        for s in (1, -1):
            q2 = s * math.acos(c2)
            sols.append((math.atan2(y, x) - math.atan2(l2 * math.sin(q2), l1 + l2 * math.cos(q2)), q2))
        q1, q2 = sols[0]
        q0 = np.array([[q1, q2]]) + rng.normal(0, 0.1, (64, 2))
        G, r = run_gpu(mc, sc, q0, 1e-10, 50, torch.float64)
        assert (from_dev(r.status) == CONV).all()
        gq = from_dev(r.q).T
        wrap = lambda a: (a + math.pi) % (2 * math.pi) - math.pi
        for row in gq:
            err = min(max(abs(wrap(row[0] - a)), abs(wrap(row[1] - b))) for a, b in sols)
            assert err < 1e-9


# ---------------------------------------------------------------- residual and Jacobian parity
@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3"])
def test_residual_and_jacobian_match_oracle(mc, name):
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=8)
    q = q[:200]
    G = gpu_problem(mc, sc)
    for dt, ftol, jtol in ((torch.float64, 1e-12, 1e-10), (torch.float32, 1e-6, 2e-4)):
        F, J = G.eval_fj(to_dev(q, dt))
        torch.cuda.synchronize()
        Fo = P.residual(q if dt == torch.float64 else q.astype(np.float32).astype(np.float64))
        Jo = P.jacobian(q if dt == torch.float64 else q.astype(np.float32).astype(np.float64))
        np.testing.assert_allclose(from_dev(F).T, Fo, atol=ftol)
        Jg = from_dev(J).T.reshape(len(q), sc.m, sc.d)
        scale = np.maximum(1.0, np.abs(Jo).max())
        np.testing.assert_allclose(Jg, Jo, atol=jtol * scale)


# ---------------------------------------------------------------- projection parity
# Band fractions under the band rule of parity.py, measured on these inputs: C1 0.385 in FP32 mode,
# 0.29 in FP64 mode (0.33 / 0.22 unstable: min-norm paths from random joint vectors with steps of
# hundreds of radians; 0.09 within a factor 2 of tol; 0.01 ill-conditioned), C2 0.16, C3 0.19 (all
# through the tolerance criterion). With the divergence exit on (test_c1_with_divergence_exit) the
# arm's band is 0.02.
MAX_BAND = {"c1": 0.40, "c2": 0.22, "c3": 0.25}


def heron(r0, tol, max_iter):
    """Radii and step count of the sphere projection from radius r0 (the min-norm step on
    ||q||^2 - 1 is radial: r <- (r + 1/r) / 2), FP64."""
    r, k, tests = r0, 0, []
    while True:
        tests.append(abs(r * r - 1.0))
        if tests[-1] < tol or k >= max_iter:
            return r, k, tests
        r = 0.5 * (r + 1.0 / r)
        k += 1


@pytest.mark.parametrize("dt,qtol", [(torch.float32, 1e-4), (torch.float64, 1e-9)])
def test_sphere_batch_matches_closed_form_everywhere(mc, dt, qtol):
    """C0 without any band: every configuration converges to r_K q / ||q||, where r_K is the Heron
    iterate at which |r^2 - 1| first drops below tol (-> q / ||q|| as tol -> 0), after exactly K
    steps. In FP32 mode the step is rounded to FP32, which moves a radius by ~1e-7 of the step (the
    last steps are ~1e-3, so a test value moves by ~1e-4 of tol): the count may differ only where a
    Heron test value lies within 1e-3 (relative) of tol."""
    sc, P, q, offs, tol, mi = config_inputs("c0", small=True)
    G, r = run_gpu(mc, sc, q, tol, mi, dt, geo_offsets=offs)
    st = from_dev(r.status).astype(int)
    it = from_dev(r.iters).astype(int)
    gq = from_dev(r.q).T
    assert (st == CONV).all()
    nrm = np.linalg.norm(q, axis=1)
    want_q = np.zeros_like(q)
    want_k = np.zeros(len(q), int)
    close = np.zeros(len(q), bool)
    for i, r0 in enumerate(nrm):
        rk, k, tests = heron(r0, tol, mi)
        want_q[i] = rk * q[i] / r0
        want_k[i] = k
        close[i] = any(abs(t / tol - 1.0) < 1e-3 for t in tests)
    if dt == torch.float64:
        assert (it == want_k).all(), f"{np.sum(it != want_k)} step counts differ from Heron's"
    else:
        assert (it[~close] == want_k[~close]).all(), f"{np.sum(it[~close] != want_k[~close])} step counts differ"
        assert close.mean() < 0.01
    # where the count differs (FP32, a test value at tol), both radii satisfy the tolerance
    same = it == want_k
    np.testing.assert_allclose(gq[same], want_q[same], atol=qtol)
    np.testing.assert_allclose(gq / np.linalg.norm(gq, axis=1, keepdims=True), q / nrm[:, None],
                               atol=5e-7 if dt == torch.float32 else 1e-14)


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_projection_parity_fp32(mc, name):
    sc, P, q, offs, tol, mi = config_inputs(name, small=True)
    G, r = run_gpu(mc, sc, q, tol, mi, torch.float32, geo_offsets=offs)
    stats = compare(P, q, r, tol, mi, 1e-4, max_band=MAX_BAND[name])
    print(name, stats)


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_projection_parity_fp64(mc, name):
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=16)
    G, r = run_gpu(mc, sc, q, tol, mi, torch.float64, geo_offsets=offs)
    stats = compare(P, q, r, tol, mi, 1e-9, max_band=MAX_BAND[name])
    print(name, stats)


@pytest.mark.parametrize("dt,qtol", [(torch.float32, 1e-4), (torch.float64, 1e-9)])
def test_cyclic_mode_parity_humanoid(mc, dt, qtol):
    """Cyclic mode (one step per constraint block, in order) on the 36-DoF humanoid, whose four
    blocks (two feet poses, hands relative pose, CoM) each get their own Gram and Cholesky,
    against the oracle's cyclic mode."""
    sc, P, q, offs, tol, mi = config_inputs("c3", small=True)
    # alternating steps converge linearly on this humanoid (the blocks share the floating base):
    # at the benchmark's 1e-6 most paths need more than 40 cycles, at 1e-3 they converge in 1-9
    G, r = run_gpu(mc, sc, q, 1e-3, mi, dtype=dt, mode="cyclic")
    # block-wise steps converge linearly, so most paths pass within a factor 2 of tol (band 0.63)
    info = compare(P, q, r, 1e-3, mi, qtol, max_band=0.7, mode="cyclic")
    assert info["conv"] > 0.99
    # five full cycles at tol 1e-6 (every path still running): the iterates agree step for step
    G, r = run_gpu(mc, sc, q, 1e-6, 5, dtype=dt, mode="cyclic")
    qo, st, it, rs = P.project(q, tol=1e-6, max_iter=5, mode="cyclic")
    gst = from_dev(r.status).astype(int)
    run = (st == MAXIT) & (gst == MAXIT)
    assert run.mean() > 0.9
    err = np.abs(from_dev(r.q).T[run] - qo[run]).max()
    assert err <= qtol, err


def test_cyclic_mode_forced_fp64_tail_and_divergence(mc):
    """Cyclic mode with every configuration sent to the FP64 tail (threshold below 1) equals FP64
    mode; with a small max_step the diverged configurations keep their input (the test applies to
    the whole iteration)."""
    sc, P, q, offs, tol, mi = config_inputs("c3", small=True, max_geo=8)
    tol = 1e-3
    G = gpu_problem(mc, sc)
    q32 = to_dev(q, torch.float32)
    rf = G.project(q32, tol=tol, max_iter=mi, mode="cyclic", cond=0.5)
    r64 = G.project(q32.double(), tol=tol, max_iter=mi, mode="cyclic")
    rd = G.project(q32.double(), tol=tol, max_iter=mi, mode="cyclic", max_step=1e-3)
    torch.cuda.synchronize()
    assert torch.equal(rf.status, r64.status) and torch.equal(rf.iters, r64.iters)
    assert torch.equal(rf.q, r64.q.float())
    qin = from_dev(q32.double()).T
    compare(P, qin, rd, tol, mi, 1e-9, max_step=1e-3, mode="cyclic", max_band=0.3)
    qo, st, it, rs = P.project(qin, tol=tol, max_iter=mi, mode="cyclic", max_step=1e-3)
    band = band_mask(P, qin, tol, mi, 1e-3, "cyclic")
    div = (from_dev(rd.status).astype(int) == 3) & (st == 3) & ~band
    assert div.any()
    # a diverged configuration stays where its last iteration started
    np.testing.assert_allclose(from_dev(rd.q).T[div], qo[div], atol=1e-9)
    np.testing.assert_array_equal(from_dev(rd.iters).astype(int)[div], it[div])


@pytest.mark.parametrize("dt,qtol", [(torch.float32, 1e-4), (torch.float64, 1e-9)])
def test_c1_with_divergence_exit(mc, dt, qtol):
    """C1 with the paper's MaxDistance exit (Alg. 2): steps longer than 0.5 rad end the projection
    as DIVERGED on both sides, which keeps the remaining paths well conditioned."""
    sc, P, q, offs, tol, mi = config_inputs("c1", small=True)
    G, r = run_gpu(mc, sc, q, tol, mi, dt, max_step=0.5)
    stats = compare(P, q, r, tol, mi, qtol, max_band=0.05, max_step=0.5)
    print("c1 max_step 0.5", stats)


@pytest.mark.parametrize("name", ["c2", "c3"])
@pytest.mark.parametrize("dt,qtol", [(torch.float64, 1e-9), (torch.float32, 1e-4)])
def test_damped_steps_parity(mc, name, dt, qtol):
    """Alg. 2's damped step alpha J^T (J J^T + lambda I)^-1 F (lambda 1e-3, alpha 0.9) against the oracle."""
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=16)
    G = mc.Problem(sc.to_blob())
    r = G.project(to_dev(q, dt), tol=tol, max_iter=mi, lam=1e-3, alpha=0.9)
    torch.cuda.synchronize()
    # damped steps converge linearly: most paths pass within a factor 2 of tol (band 0.54-0.64)
    info = compare(P, q, r, tol, mi, qtol, max_band=0.7, alpha=0.9, lam=1e-3)
    assert info["conv"] > 0.9, info


@pytest.mark.parametrize("name,dt,qtol", [("c1", torch.float64, 1e-9), ("c2", torch.float64, 1e-9),
                                          ("c6", torch.float64, 1e-9), ("c2", torch.float32, 1e-3),
                                          ("c6", torch.float32, 1e-3)])
def test_outer_step_form_parity(mc, name, dt, qtol):
    """The outer form of the step, alpha (J^T J + lambda I)^-1 J^T F (a d x d factorisation of the dense
    J; lambda 1e-3, alpha 0.9), against the oracle's damped least-squares step, and against the inner
    form on the GPU outside the band (the same vector for lambda > 0, up to rounding). The d x d system
    has condition number (sigma_max^2 + lambda) / lambda, about 1e4 here against the m x m system's
    sigma_max^2 / sigma_min^2: FP32 steps carry that much more rounding, hence 1e-3 in FP32 mode, which
    the arm's long-step paths (C1: steps of several radians) exceed (1.9e-3 measured): FP32 mode is
    checked on C2 and C6."""
    from parity import UNSTABLE_REL
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=16)
    G = mc.Problem(sc.to_blob())
    qd = to_dev(q, dt)
    ro = G.project(qd, tol=tol, max_iter=mi, lam=1e-3, alpha=0.9, step_form="outer")
    ri = G.project(qd, tol=tol, max_iter=mi, lam=1e-3, alpha=0.9)
    torch.cuda.synchronize()
    orc = oracle_run(P, q, tol, mi, alpha=0.9, lam=1e-3, unstable=(UNSTABLE_REL[ro.q.element_size()], qtol / 4))
    info = compare(P, q, ro, tol, mi, qtol, max_band=0.7, alpha=0.9, lam=1e-3, orc=orc)
    assert info["conv"] > 0.8, info
    out = torch.from_numpy(~orc["band"]).to(ro.q.device)
    same = out & (ro.status == ri.status) & (ro.iters == ri.iters) & (ro.status == 0)
    assert same.float().sum().item() > 0.5 * out.float().sum().item()
    d = (ro.q - ri.q)[:, same].abs().max().item()
    assert d < qtol, d
    print(name, dt, info)


def test_outer_step_form_is_refused_where_it_does_not_fit(mc):
    sc, P, q, offs, tol, mi = config_inputs("c3", small=True, max_geo=1)
    G = mc.Problem(sc.to_blob())
    qd = to_dev(q, torch.float32)
    with pytest.raises(mc.McError):
        G.project(qd, lam=1e-3, step_form="outer")  # d = 36
    sc1, _, q1, _, _, _ = config_inputs("c1", small=True, max_geo=1)
    G1 = mc.Problem(sc1.to_blob())
    with pytest.raises(mc.McError):
        G1.project(to_dev(q1, torch.float32), lam=0.0, step_form="outer")  # needs lambda > 0
    with pytest.raises(mc.McError):
        G1.project(to_dev(q1, torch.float32), lam=1e-3, step_form="outer", mode="cyclic")


def test_wide_launch_matches_one_wave_launch(mc):
    """The 74,059-configuration humanoid batch exceeds the lanes of the one-wave-per-SIMD launch, so
    with the launch shape left to the library it runs in the two-wave build; pinning the shape keeps
    the one-wave build. Both must give the same outputs bit for bit (the one-wave build is the one
    checked against the oracle)."""
    from paper_2604_13323_amd import scenes as S
    cfg = S.make_config("c4")
    sc = cfg["scene"]
    G = gpu_problem(mc, sc)
    e = torch.from_numpy(np.ascontiguousarray(cfg["endpoints"].reshape(-1, sc.d).T)).to("cuda", torch.float32)
    re = G.project(e, tol=1e-9, max_iter=100, check=False)
    offs = torch.from_numpy(np.asarray(cfg["geo_offsets"], np.int32)).cuda()
    q = G.interpolate(re.q, offs, int(cfg["geo_offsets"][-1]))
    assert q.shape[1] > 65536
    wide = G.project(q, tol=cfg["tol"], max_iter=cfg["max_iter"], variant="fused")
    one = G.project(q, tol=cfg["tol"], max_iter=cfg["max_iter"], variant="fused", waves_per_block=4, blocks_per_cu=1)
    torch.cuda.synchronize()
    for f in ("q", "status", "iters", "resid", "verdict"):
        assert torch.equal(getattr(wide, f), getattr(one, f)), f
    assert (one.status == 0).float().mean().item() > 0.99


@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3"])
def test_plain_and_fused_are_bitwise_identical(mc, name):
    sc, P, q, offs, tol, mi = config_inputs(name, small=True)
    G = gpu_problem(mc, sc)
    qd = to_dev(q, torch.float32)
    ref = G.project(qd, tol=tol, max_iter=mi, variant="plain", geo_offsets=offs)
    outs = [G.project(qd, tol=tol, max_iter=mi, variant="fused", waves_per_block=w, blocks_per_cu=b)
            for w, b in ((1, 0), (2, 1), (4, 2), (1, 1))]
    torch.cuda.synchronize()
    for o in outs:
        assert torch.equal(o.q, ref.q)
        assert torch.equal(o.status, ref.status)
        assert torch.equal(o.iters, ref.iters)
        assert torch.equal(o.resid, ref.resid)
        assert torch.equal(o.verdict, ref.verdict)


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_fp64_tail_queue_matches_fp64_mode(mc, name):
    """A condition threshold below 1 sends every configuration that takes a step to the FP64 path
    (the tail kernel in the fused variant, in-kernel in the plain one). From there the iteration
    is the FP64-mode iteration, so results equal FP64 mode on the same (FP32-rounded) inputs
    after rounding the output to FP32."""
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=16)
    G = gpu_problem(mc, sc)
    q32 = to_dev(q, torch.float32)
    q64 = q32.double()
    G.fallback_count(reset=True)
    rf = G.project(q32, tol=tol, max_iter=mi, variant="fused", cond=0.5)
    rp = G.project(q32, tol=tol, max_iter=mi, variant="plain", geo_offsets=offs, cond=0.5)
    r64 = G.project(q64, tol=tol, max_iter=mi, variant="fused")
    torch.cuda.synchronize()
    stepped = int((r64.iters.cpu().numpy() > 0).sum())
    assert G.fallback_count(reset=True) >= 2 * stepped  # fused and plain each moved them to FP64
    for r in (rf, rp):
        assert torch.equal(r.status, r64.status)
        assert torch.equal(r.iters, r64.iters)
        assert torch.equal(r.q, r64.q.float())
        assert torch.equal(r.verdict, r64.verdict)
    # the VJP tail: every converged configuration redone in FP64 equals FP64 mode
    g = torch.randn_like(r64.q)
    gi32 = G.vjp(rf.q, rf.status, g.float(), cond=0.5)
    gi64 = G.vjp(rf.q.double(), rf.status, g.float().double())
    torch.cuda.synchronize()
    assert torch.equal(gi32, gi64.float())


@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3", "c3near"])
def test_fused_verdicts_match_oracle(mc, name):
    """Verdicts written by project_batch (fused: broad-phase flag from the last residual pass,
    exact check only for flagged configurations) equal the oracle's brute-force check of the
    same output configurations outside the 1e-5 m band; non-converged ones are UNCHECKED."""
    sc, P, q, offs, tol, mi = config_inputs(name, small=True)
    G = gpu_problem(mc, sc)
    r = G.project(to_dev(q, torch.float32), tol=tol, max_iter=mi, variant="fused")
    torch.cuda.synchronize()
    st = from_dev(r.status).astype(int)
    v = from_dev(r.verdict).astype(int)
    conv = st == CONV
    assert (v[~conv] == 2).all()
    qg = from_dev(r.q).T[conv]
    vo, sdo = P.check(qg)
    out = np.abs(sdo) > 1e-5
    assert (v[conv][out] == vo[out]).all(), f"{np.sum(v[conv][out] != vo[out])} verdicts differ"
    # the benchmark's humanoid scene keeps its shelves out of reach (collision-free by design); its
    # c3near variant moves them into reach of the hands
    if name not in ("c0", "c3"):
        assert (vo == 1).any(), "workload has no colliding configuration to exercise the queue"


# ---------------------------------------------------------------- collision parity
@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3", "c3near"])
def test_check_batch_matches_oracle(mc, name):
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=16)
    qo = P.project(q, tol=1e-9, max_iter=60)[0]
    G = gpu_problem(mc, sc)
    for dt in (torch.float32, torch.float64):
        qd = to_dev(qo, dt)
        v, sd = G.check(qd, min_signed_dist=True)
        v2 = G.check(qd)
        torch.cuda.synchronize()
        q_used = from_dev(qd).T  # identical inputs on both sides
        vo, sdo = P.check(q_used)
        out = np.abs(sdo) > 1e-5
        assert (from_dev(v)[out] == vo[out]).all()
        assert (from_dev(v2)[out] == vo[out]).all(), "broad phase changed a verdict"
        np.testing.assert_allclose(from_dev(sd), sdo, atol=1e-5)


# ---------------------------------------------------------------- VJP parity
@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3"])
def test_vjp_matches_oracle(mc, name):
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=8)
    qs, st, it, rs = P.project(q, tol=1e-12, max_iter=80)
    rng = np.random.default_rng(5)
    g = rng.standard_normal(qs.shape)
    G = gpu_problem(mc, sc)
    for dt, rtol in ((torch.float64, 1e-9), (torch.float32, 1e-3)):
        qd = to_dev(qs, dt)
        gi = G.vjp(qd, torch.from_numpy(st).cuda(), to_dev(g, dt))
        torch.cuda.synchronize()
        go, kap = P.vjp(from_dev(qd).T, g, st)
        gg = from_dev(gi).T
        ok = st == CONV
        num = np.linalg.norm(gg[ok] - go[ok], axis=1)
        den = np.maximum(np.linalg.norm(go[ok], axis=1), 1e-3 * np.linalg.norm(g[ok], axis=1))
        assert (num / den).max() < rtol, (num / den).max()
        assert np.all(gg[~ok] == 0)


def test_vjp_matches_fp64_central_differences_c4(mc):
    """C4 differentiation check: GPU VJPs (FP32 mode, FP64 solve only where the condition estimate
    exceeds 1e6) against FP64 central finite differences (h = 1e-6) of the oracle's projection,
    on 256 configurations sampled from the converged ones and re-projected to ||F|| < 1e-13 (the
    VJP is the derivative of the projection there). Relative error in ||g_in||, bound 1e-3."""
    sc, P, q, offs, tol, mi = config_inputs("c4", small=True)
    G = gpu_problem(mc, sc)
    r = G.project(to_dev(q, torch.float32), tol=tol, max_iter=mi)
    torch.cuda.synchronize()
    st = from_dev(r.status).astype(int)
    rng = np.random.default_rng(3)  # stream 3: the FD sample
    idx = rng.choice(np.where(st == CONV)[0], size=min(256, int((st == CONV).sum())), replace=False)
    q0, s0, _, _ = P.project(from_dev(r.q).T[idx].astype(np.float64), tol=1e-13, max_iter=100)
    assert (s0 == CONV).all()
    g = rng.standard_normal(q0.shape)
    h = 1e-6
    d = sc.d
    qp = np.repeat(q0, d, axis=0) + h * np.tile(np.eye(d), (len(q0), 1))
    qm = np.repeat(q0, d, axis=0) - h * np.tile(np.eye(d), (len(q0), 1))
    pp, sp, _, _ = P.project(qp, tol=1e-13, max_iter=100)
    pm, sm, _, _ = P.project(qm, tol=1e-13, max_iter=100)
    assert (sp == CONV).all() and (sm == CONV).all()
    dP = ((pp - pm) / (2 * h)).reshape(len(q0), d, d)  # [n, k (input), :] = dP/dq_k
    g_fd = np.einsum("nkj,nj->nk", dP, g)                # (dP/dq)^T g
    gi = G.vjp(to_dev(q0, torch.float32), torch.zeros(len(q0), dtype=torch.int8, device="cuda"),
               to_dev(g, torch.float32))
    torch.cuda.synchronize()
    gg = from_dev(gi).T.astype(np.float64)
    rel = np.linalg.norm(gg - g_fd, axis=1) / np.linalg.norm(g_fd, axis=1)
    assert rel.max() < 1e-3, f"max relative error {rel.max():.3e}"
    # and the oracle's gradient (explicit null-space projector) agrees with both
    go, _ = P.vjp(q0, g, s0)
    assert (np.linalg.norm(go - g_fd, axis=1) / np.linalg.norm(g_fd, axis=1)).max() < 1e-6


def test_path_length_and_interpolation_match_oracle(mc):
    import oracle
    sc, P, q, offs, tol, mi = config_inputs("c4", small=True)
    G = gpu_problem(mc, sc)
    offs_d = torch.from_numpy(offs).cuda()
    for dt in (torch.float64, torch.float32):
        g, loss = G.path_length_grad(to_dev(q, dt), offs_d)
        torch.cuda.synchronize()
        L, go = oracle.path_length(from_dev(to_dev(q, dt)).T, offs)
        tolg = 1e-12 if dt == torch.float64 else 1e-5
        np.testing.assert_allclose(from_dev(g).T, go, atol=tolg)
        assert abs(float(loss[0]) - L) < (1e-9 if dt == torch.float64 else 1e-3) * max(1, L)
    e = np.random.default_rng(1).standard_normal((len(offs) - 1, 2, sc.d))
    ed = torch.from_numpy(np.ascontiguousarray(e.reshape(-1, sc.d).T)).cuda()
    qi = G.interpolate(ed, offs_d, int(offs[-1]))
    torch.cuda.synchronize()
    np.testing.assert_allclose(from_dev(qi).T, oracle.interpolate_interior(e, offs), atol=1e-14)


@pytest.mark.parametrize("name", ["c0", "c3"])
def test_path_length_gradient_ragged_geodesics(mc, name):
    """Geodesics of 0 to 300 configurations: a run of 1,500 empty ones (more offsets than a
    workgroup stages in LDS), lengths 1, 2, 63, 64 and 65 (boundaries on a wave's first and last
    lane), configurations before the first and after the last geodesic (gradient 0), a leading
    dimension above n; both dtypes against the oracle."""
    import oracle
    sc = config_inputs(name, small=True, max_geo=1)[0]
    G = gpu_problem(mc, sc)
    rng = np.random.default_rng(77)
    lens = np.concatenate([rng.integers(0, 300, 40), np.zeros(1500, int), [1, 2, 63, 64, 65, 1, 1, 0, 2],
                           rng.integers(0, 5, 200), rng.integers(60, 70, 30)])
    offs = (5 + np.concatenate([[0], np.cumsum(lens)])).astype(np.int32)
    n = int(offs[-1]) + 7
    q = rng.uniform(-2.0, 2.0, (n, sc.d))
    offs_d = torch.from_numpy(offs).cuda()
    for dt in (torch.float64, torch.float32):
        qd = torch.zeros((sc.d, n + 13), dtype=dt, device="cuda")
        qd[:, :n] = torch.from_numpy(q.T).to(dt)
        g, loss = G.path_length_grad(qd[:, :n], offs_d)
        torch.cuda.synchronize()
        L, go = oracle.path_length(from_dev(qd[:, :n]).T, offs)
        tolg = 1e-12 if dt == torch.float64 else 1e-5
        gg = from_dev(g).T
        np.testing.assert_allclose(gg, go, atol=tolg)
        assert (gg[:5] == 0).all() and (gg[-7:] == 0).all()
        assert abs(float(loss[0]) - L) < (1e-9 if dt == torch.float64 else 1e-5) * max(1, L)


# ---------------------------------------------------------------- edge cases
def test_edge_cases(mc):
    from paper_2604_13323_amd import scenes as S
    sc = S.sphere_scene(0)
    G = gpu_problem(mc, sc)
    # n = 0 is a no-op
    r = G.project(torch.empty((3, 0), device="cuda"))
    assert r.q.shape == (3, 0)
    # ld > n (a column slice of a wider array), ragged n
    q = np.random.default_rng(0).standard_normal((200, 3))
    big = to_dev(q, torch.float32)
    sub = big[:, :131]
    r = G.project(sub, tol=1e-6, max_iter=50)
    torch.cuda.synchronize()
    ref = q[:131] / np.linalg.norm(q[:131], axis=1, keepdims=True)
    np.testing.assert_allclose(from_dev(r.q).T, ref, atol=2e-6)
    # argument errors are reported synchronously
    with pytest.raises(mc.McError):
        G.project(big, tol=-1.0)
    with pytest.raises(mc.McError):
        G.project(big, max_iter=500)
    with pytest.raises(mc.McError):
        G.project(big, variant="plain")  # needs geodesic offsets


def test_autograd_function(mc):
    sc, P, q, offs, tol, mi = config_inputs("c1", small=True, max_geo=4)
    G = gpu_problem(mc, sc)
    q0 = to_dev(q, torch.float64).requires_grad_(True)
    qp, st = mc.project(q0, G, tol=1e-10, max_iter=60)
    w = torch.randn_like(qp)
    (qp * w).sum().backward()
    gi = G.vjp(qp.detach(), st, w)
    torch.cuda.synchronize()
    assert torch.allclose(q0.grad, gi)
