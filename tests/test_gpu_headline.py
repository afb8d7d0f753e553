"""GPU parity on the paths the benchmark's humanoid batch takes, against the FP64 oracle:
the full 65,536-configuration batch in the autotuned launch shape the benchmark times, the same
batch with lanes refilled from the work queue, the exact-check tail on long and short queues in a
scene whose obstacles are within reach (hits), the per-geodesic success flags, the condition
estimate that decides the FP64 fallback, the autotuner, and outputs with a leading dimension
larger than the batch."""
import numpy as np
import pytest

import oracle

from parity import CONV, UNSTABLE_REL, compare, config_inputs, from_dev, oracle_run, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mc():
    import paper_2604_13323_amd as M
    M.lib()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return M


@pytest.fixture(scope="module")
def headline(mc):
    """The benchmark's humanoid batch (2,048 geodesics x 32 = 65,536 configurations), endpoints
    projected by the oracle, and the oracle's projection of every configuration."""
    sc, P, q, offs, tol, mi = config_inputs("c3", small=False)
    assert len(q) == 65536
    return dict(sc=sc, P=P, q=q, offs=offs, tol=tol, mi=mi, orc=oracle_run(P, q, tol, mi, unstable=(UNSTABLE_REL[4], 2.5e-5)),
                G=mc.Problem(sc.to_blob()), q32=to_dev(q, torch.float32))


def test_headline_batch_autotuned_matches_oracle(headline):
    """All 65,536 configurations in the launch shape the benchmark uses: the library's autotuner
    picks it (every candidate must reproduce the others bit for bit) and the auto variant runs it."""
    h = headline
    G = h["G"]
    best, table = G.autotune(h["q32"], reps=2, tol=h["tol"], max_iter=h["mi"])
    assert G.tuned_shape() == best
    r = G.project(h["q32"], tol=h["tol"], max_iter=h["mi"])  # variant auto: the tuned shape
    torch.cuda.synchronize()
    stats = compare(h["P"], h["q"], r, h["tol"], h["mi"], 1e-4, max_band=0.3, orc=h["orc"])
    print("headline", best, stats)
    h["tuned_result"] = r


def test_headline_batch_with_lane_refill_matches_oracle(headline):
    """One wave per workgroup and one workgroup per CU: 256 x 64 = 16,384 lanes for 65,536
    configurations, so every lane takes about three more configurations from the work queue."""
    h = headline
    G = h["G"]
    r = G.project(h["q32"], tol=h["tol"], max_iter=h["mi"], variant="fused", waves_per_block=1, blocks_per_cu=1)
    torch.cuda.synchronize()
    taken = G.queue_counts()[0]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    assert taken >= 65536 - n_cu * 64, taken
    stats = compare(h["P"], h["q"], r, h["tol"], h["mi"], 1e-4, max_band=0.3, orc=h["orc"])
    print("refill", taken, stats)
    ref = h.get("tuned_result")
    if ref is not None:
        for f in ("q", "status", "iters", "resid", "verdict"):
            assert torch.equal(getattr(r, f), getattr(ref, f)), f


def near_scene(small):
    sc, P, q, offs, tol, mi = config_inputs("c3near", small=small)
    return sc, P, q, offs, tol, mi


def check_verdicts(P, r):
    """Verdicts of project_batch against the oracle's brute force on the GPU's own output
    configurations (identical inputs), outside the 1e-5 m band; UNCHECKED where not converged."""
    st = from_dev(r.status).astype(int)
    v = from_dev(r.verdict).astype(int)
    conv = st == CONV
    assert (v[~conv] == 2).all()
    vo, sdo = P.check(from_dev(r.q).T[conv])
    out = np.abs(sdo) > 1e-5
    bad = v[conv][out] != vo[out]
    assert bad.sum() == 0, f"{bad.sum()} verdicts differ from the oracle"
    return vo, sdo


def test_long_exact_check_queue_with_hits_matches_oracle(mc):
    """8,192 humanoid configurations with shelf slabs in reach of the hands: more than 4,096
    converged configurations have a link near the obstacles, so the exact-check tail takes its
    long-queue path (4 lanes per configuration); most of them collide."""
    sc, P, q, offs, tol, mi = near_scene(small=False)
    G = mc.Problem(sc.to_blob())
    r = G.project(to_dev(q, torch.float32), tol=tol, max_iter=mi, variant="fused")
    torch.cuda.synchronize()
    queued = G.queue_counts()[3]
    assert queued > 4096, queued
    vo, _ = check_verdicts(P, r)
    assert vo.mean() > 0.3, vo.mean()
    compare(P, q, r, tol, mi, 1e-4, max_band=0.3)
    # check_batch on the same outputs: its broad phase queues as many, and the long-queue tail
    # gives the fused step's verdicts on the converged ones
    v = G.check(r.q)
    torch.cuda.synchronize()
    assert G.queue_counts()[3] >= queued
    conv = r.status == CONV
    assert torch.equal(v[conv], r.verdict[conv])


def test_short_exact_check_queue_plain_and_check_batch_with_hits(mc):
    """1,024 configurations of the same scene: a short queue (one wave per configuration, links split
    over up to 4 waves); the plain variant's in-line exact check and check_batch agree with it and
    with the oracle."""
    sc, P, q, offs, tol, mi = near_scene(small=True)
    G = mc.Problem(sc.to_blob())
    qd = to_dev(q, torch.float32)
    r = G.project(qd, tol=tol, max_iter=mi, variant="fused")
    torch.cuda.synchronize()
    queued = G.queue_counts()[3]
    assert 0 < queued <= 4096, queued
    vo, sdo = check_verdicts(P, r)
    assert vo.mean() > 0.3
    rp = G.project(qd, tol=tol, max_iter=mi, variant="plain", geo_offsets=offs)
    torch.cuda.synchronize()
    assert torch.equal(rp.verdict, r.verdict) and torch.equal(rp.q, r.q)
    for dt in (torch.float32, torch.float64):
        qc = r.q.to(dt)
        v = G.check(qc)
        v2, sd = G.check(qc, min_signed_dist=True)
        torch.cuda.synchronize()
        vo2, sdo2 = P.check(from_dev(qc).T)
        out = np.abs(sdo2) > 1e-5
        assert (from_dev(v)[out] == vo2[out]).all()
        assert (from_dev(v2)[out] == vo2[out]).all()
        np.testing.assert_allclose(from_dev(sd), sdo2, atol=1e-5)


def test_geo_ok_is_the_and_over_each_geodesic(mc):
    """geo_ok[g] = 1 exactly when every configuration of geodesic g converged and is collision-free,
    compared with the oracle's statuses and its verdicts on the GPU's output configurations, on the
    geodesics with no configuration whose status is uncertain (a band criterion other than the
    tolerance one, which can move the step count but not the convergence) or whose verdict lies in
    the 1e-5 m band."""
    sc, P, q, offs, tol, mi = near_scene(small=True)
    G = mc.Problem(sc.to_blob())
    r = G.project(to_dev(q, torch.float32), tol=tol, max_iter=mi, geo_offsets=offs, geo_ok=True)
    torch.cuda.synchronize()
    o = oracle_run(P, q, tol, mi)
    vo, sdo = P.check(from_dev(r.q).T)
    ok_cfg = (o["status"] == CONV) & (vo == 0)
    unsure = np.abs(sdo) <= 1e-5
    for k, m in o["parts"].items():
        if k != "near_tol":
            unsure |= m
    go = from_dev(r.geo_ok).astype(int)
    n_cmp = 0
    for g in range(len(offs) - 1):
        a, b = offs[g], offs[g + 1]
        if unsure[a:b].any():
            continue
        n_cmp += 1
        assert go[g] == int(ok_cfg[a:b].all()), g
    assert n_cmp >= 8 and 0 < go.sum() < len(go), (n_cmp, go.sum())


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_condition_estimate_matches_oracle(mc, name):
    """kappa_est = (max L_ii / min L_ii)^2 of the kernels' factorisation of J J^T against the
    oracle's FP64 Cholesky at the same configurations: FP64 mode to 1e-9 relative; FP32 mode within
    what FP32 kinematics and Gram rounding allow. The Gram entries carry a few units of FP32 rounding
    relative to ||J||^2, and a pivot of the factorisation, at least sigma_min(J)^2, moves by that
    much, so the relative error of kappa_est is bounded by a multiple of kappa_2 = (sigma_max /
    sigma_min)^2 of J, which can be far larger than kappa_est itself on a badly scaled Gram: 1e-6
    kappa_2 + 1e-4. The FP64-fallback decision at 1e6 agrees outside a factor 4 around the
    threshold."""
    sc, P, q, offs, tol, mi = config_inputs(name, small=True, max_geo=16)
    G = mc.Problem(sc.to_blob())
    for dt in (torch.float64, torch.float32):
        qd = to_dev(q, dt)
        k = from_dev(G.condition(qd))
        torch.cuda.synchronize()
        ke, k2 = P.kappa_est(from_dev(qd).T)
        fin = np.isfinite(ke)
        if dt == torch.float64:
            # both factorise in FP64 by different operation orders: relative rounding ~ 1e-16 kappa
            rel = np.abs(k[fin] / ke[fin] - 1.0)
            assert (rel <= 1e-9 + 1e-15 * ke[fin]).all(), rel.max()
        else:
            ok = fin & (ke < 1e5)
            rel = np.abs(k[ok] / ke[ok] - 1.0)
            worst = np.argmax(rel - 1e-6 * k2[ok])
            assert (rel <= 1e-6 * k2[ok] + 1e-4).all(), (rel[worst], ke[ok][worst], k2[ok][worst])
            sure = fin & ((ke < 0.25e6) | (ke > 4e6))
            assert ((k[sure] > 1e6) == (ke[sure] > 1e6)).all()
        print(name, dt, "kappa_est range", np.nanmin(ke), np.nanmax(ke[fin]), "above 1e6:", int((ke > 1e6).sum()))


def test_strided_outputs_of_vjp_and_path_gradient(mc):
    """A column slice of a wider array (leading dimension 200 > n = 131): the VJP and the path-length
    gradient are written with the input's leading dimension and equal the contiguous results."""
    sc, P, q, offs, tol, mi = config_inputs("c3", small=True, max_geo=8)
    G = mc.Problem(sc.to_blob())
    r = G.project(to_dev(q, torch.float32), tol=1e-6, max_iter=40)
    big = torch.zeros((sc.d, 200), dtype=torch.float32, device="cuda")
    big[:, :131] = r.q[:, :131]
    gbig = torch.randn((sc.d, 200), dtype=torch.float32, device="cuda")
    sub, gsub = big[:, :131], gbig[:, :131]
    assert sub.stride(0) == 200
    gi = G.vjp(sub, r.status[:131].contiguous(), gsub)
    gi_ref = G.vjp(sub.contiguous(), r.status[:131].contiguous(), gsub.contiguous())
    offs_d = torch.tensor([0, 64, 131], dtype=torch.int32, device="cuda")
    pg, _ = G.path_length_grad(sub, offs_d)
    pg_ref, _ = G.path_length_grad(sub.contiguous(), offs_d)
    torch.cuda.synchronize()
    assert gi.stride(0) == 200 and pg.stride(0) == 200
    assert torch.equal(gi, gi_ref)
    assert torch.equal(pg, pg_ref)


def test_autotuner_result_is_used_by_the_auto_variant(mc):
    sc, P, q, offs, tol, mi = config_inputs("c2", small=True)
    G = mc.Problem(sc.to_blob())
    assert G.tuned_shape() is None
    qd = to_dev(q, torch.float32)
    best, table = G.autotune(qd, reps=2, tol=tol, max_iter=mi)
    assert len(table) >= 7 and all(ms > 0 for _, ms in table)
    assert G.tuned_shape() == best and G.tuned_shape(torch.float64) is None
    ra = G.project(qd, tol=tol, max_iter=mi)
    rb = G.project(qd, tol=tol, max_iter=mi, variant="fused", waves_per_block=best["waves_per_block"],
                   blocks_per_cu=best["blocks_per_cu"])
    torch.cuda.synchronize()
    for f in ("q", "status", "iters", "resid", "verdict"):
        assert torch.equal(getattr(ra, f), getattr(rb, f)), f
    with pytest.raises(mc.McError):
        G.project(qd, lanes_per_config=3)


class _Sub:
    """The columns idx of a ProjectResult (what compare reads)."""

    def __init__(self, r, idx):
        ix = torch.as_tensor(idx, device=r.q.device)
        self.q = r.q[:, ix]
        self.status = r.status[ix]
        self.iters = r.iters[ix]
        self.resid = r.resid[ix]
        self.verdict = r.verdict[ix]


FULL = {"c1": (0.45, 131072), "c2": (0.25, 1078723), "c5": (0.30, 65536), "c6": (0.25, 131072)}


@pytest.mark.parametrize("name", ["c1", "c2", "c5", "c6"])
def test_full_size_batches_sampled_against_oracle(mc, name):
    """The other benchmark batches at full size through the path the benchmark times (fused variant,
    the library's launch shape: lanes refill from the work queue, C1's and C2's uneven step counts
    balance over it), compared with the oracle on 2,048 sampled configurations under the band rule."""
    from paper_2604_13323_amd import scenes as S
    import bench
    cfg = S.make_config(name)
    sc = cfg["scene"]
    G = mc.Problem(sc.to_blob())
    if "q" in cfg:
        q = np.asarray(cfg["q"], np.float64)
    else:
        qd, _, _ = bench.build_batch(G, cfg, torch)
        q = from_dev(qd).T
    max_band, n_want = FULL[name]
    assert len(q) == n_want
    r = G.project(to_dev(q, torch.float32), tol=cfg["tol"], max_iter=cfg["max_iter"], variant="fused")
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng([len(q), 9]).choice(len(q), size=2048, replace=False))
    P = oracle.Problem(sc.to_blob())
    qs = from_dev(to_dev(q[idx], torch.float32)).T  # the inputs the GPU saw
    sub = _Sub(r, idx)
    stats = compare(P, qs, sub, cfg["tol"], cfg["max_iter"], 1e-4, max_band=max_band)
    # collision verdicts of the sampled converged configurations (the long-queue path of the
    # exact-check tail) against the oracle's brute force at the GPU's outputs, outside the 1e-5 m band
    conv = from_dev(sub.status).astype(int) == CONV
    vo, sdo = P.check(from_dev(sub.q).T[conv])
    vg = from_dev(sub.verdict).astype(int)[conv]
    out = np.abs(sdo) > 1e-5
    assert (vg[out] == vo[out]).all(), f"{int((vg[out] != vo[out]).sum())} verdicts differ"
    print(name, len(q), stats, "hits", int(vo.sum()), "queued", G.queue_counts()[3])


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_exact_check_lane_groups_give_the_same_verdicts(mc, name):
    """The exact-check tail with every lane-group size forced (a wave, 16, 8, 4, 2 and 1 lanes per
    configuration; the 36-DoF family keeps at least 4) gives bit-identical verdicts, in check_batch
    and in the fused projection, and they match the oracle outside the 1e-5 m band."""
    sc, P, q, offs, tol, mi = config_inputs(name, small=True)
    G = mc.Problem(sc.to_blob())
    qd = to_dev(q, torch.float32)
    ref = G.project(qd, tol=tol, max_iter=mi, variant="fused")
    vref = G.check(ref.q)
    torch.cuda.synchronize()
    assert G.queue_counts()[3] > 0
    for lanes in (64, 16, 8, 4, 2, 1):
        G.set_check_lanes(lanes)
        r = G.project(qd, tol=tol, max_iter=mi, variant="fused")
        v = G.check(ref.q)
        torch.cuda.synchronize()
        assert torch.equal(r.verdict, ref.verdict), lanes
        assert torch.equal(v, vref), lanes
    G.set_check_lanes(0)
    with pytest.raises(mc.McError):
        G.set_check_lanes(3)
    conv = from_dev(ref.status).astype(int) == CONV
    vo, sdo = P.check(from_dev(ref.q).T[conv])
    out = np.abs(sdo) > 1e-5
    assert (from_dev(vref).astype(int)[conv][out] == vo[out]).all()


def test_autotuner_picks_the_check_lane_groups_on_a_long_queue(mc):
    """On the 7-DoF arm batch at full size almost every configuration reaches the exact check, so the
    autotuner's second stage times lane groups of 1, 2, 4, 8 and 16 for it, keeps the fastest in the problem
    and reports it; later calls give the same outputs as the untuned call. A short queue (the humanoid
    batch) leaves the choice untuned."""
    from paper_2604_13323_amd import scenes as S
    import bench
    cfg = S.make_config("c1")
    G = mc.Problem(cfg["scene"].to_blob())
    if "q" in cfg:
        q = to_dev(np.asarray(cfg["q"], np.float64), torch.float32)
    else:
        q, _, _ = bench.build_batch(G, cfg, torch)
    kw = dict(tol=cfg["tol"], max_iter=cfg["max_iter"])
    ref = G.project(q, variant="fused", **kw)
    torch.cuda.synchronize()
    assert G.queue_counts()[3] > 16 * 256
    best, table = G.autotune(q, reps=2, **kw)
    assert best["check_lanes"] in (1, 2, 4, 8, 16), best
    assert G.tuned_shape() == best
    r = G.project(q, **kw)
    torch.cuda.synchronize()
    for f in ("q", "status", "iters", "resid", "verdict"):
        assert torch.equal(getattr(r, f), getattr(ref, f)), f
    sc3, P3, q3, offs3, tol3, mi3 = config_inputs("c3", small=True)
    G3 = mc.Problem(sc3.to_blob())
    best3, _ = G3.autotune(to_dev(q3, torch.float32), reps=1, tol=tol3, max_iter=mi3)
    assert best3["check_lanes"] == 0
