#!/usr/bin/env python3
"""Benchmark of the batched manifold projection on one MI355X.

Headline: converged projections/s on the 36-DoF humanoid batch (65,536 configurations =
2,048 geodesics x 32 interior interpolants between projected endpoints, tol 1e-6, at most
40 Newton steps, collision check against 500 shelf spheres fused into the step), with the
fused persistent work-queue kernel. Also measured: the plain per-geodesic launch on the same
batch, and fwd+VJP/s on the differentiation batch (2,048 geodesics of 8..64 interpolants:
projection + path-length gradient + VJP).

A "step" is one pass of the whole hot path over the batch, inputs resident in HBM. Timing:
HIP events on the stream the kernels run on, W untimed warm-up steps, then K timed steps.
Prints one JSON line (last line of stdout).
"""
from __future__ import annotations

import argparse
import hashlib
import glob
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3         # MI355X published FP32 vector peak (counts packed FP32 FMAs)
PEAK_NONPACKED_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz (non-packed FP32 and FP64)
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PROJECTION_SOURCES = ("common.hpp", "kin.hpp", "kernels.hpp", "ops.hpp", "ops_impl.hpp", "fam_humanoid36_f32_persistent.hip")


def source_hash() -> str:
    """Hash of the sources the humanoid projection kernel is compiled from (its counter-based traffic
    figure is reported only while they are unchanged)."""
    h = hashlib.sha256()
    for name in PROJECTION_SOURCES:
        with open(os.path.join(ROOT, "paper_2604_13323_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


STEP_MEDIANS = {}


def timed(fn, steps, warmup, torch, name=None):
    """Mean ms per step over `steps` steps after `warmup` untimed ones (HIP events on the current
    stream, which the library launches on); with a name, the median of the per-step times is kept
    in STEP_MEDIANS as well."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for k in range(steps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    if name:
        STEP_MEDIANS[name] = float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))
    return ev[0].elapsed_time(ev[steps]) / steps  # ms per step


def build_batch(G, cfg, torch):
    """Project the geodesic endpoints (library, untimed) and interpolate the interior points."""
    sc = cfg["scene"]
    E = cfg["endpoints"].reshape(-1, sc.d)  # rows 2g, 2g+1 = the two ends of geodesic g
    e = torch.from_numpy(np.ascontiguousarray(E.T)).to("cuda", torch.float32)
    re = G.project(e, tol=1e-9, max_iter=100, check=False)
    offs = torch.from_numpy(np.asarray(cfg["geo_offsets"], np.int32)).cuda()
    n = int(cfg["geo_offsets"][-1])
    q = G.interpolate(re.q, offs, n)
    torch.cuda.synchronize()
    return q, offs, re


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, max_configs: int, runs: int = 3):
    """The FP64 oracle on the same workload recipe (its own endpoint projection and interpolation):
    wall clock of projection + brute-force check over the sample, median of `runs` runs."""
    import oracle
    sc = cfg["scene"]
    P = oracle.Problem(sc.to_blob())
    offs = np.asarray(cfg["geo_offsets"], np.int32)
    n_geo = len(offs) - 1
    per = int(offs[1] - offs[0])
    g_take = max(1, min(n_geo, max_configs // max(per, 1)))
    offs = offs[:g_take + 1]
    e = cfg["endpoints"][:g_take].reshape(-1, sc.d)
    qe = P.project(e, tol=1e-9, max_iter=100)[0]
    q = oracle.interpolate_interior(qe.reshape(-1, 2, sc.d), offs)
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        qo, st, it, rs = P.project(q, tol=cfg["tol"], max_iter=cfg["max_iter"])
        conv = st == 0
        v, _ = P.check(qo[conv])
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    # one thread on the first 2,048 configurations of the same sample
    q1 = q[:2048]
    t1 = time.perf_counter()
    qo1, st1, _, _ = P.project(q1, tol=cfg["tol"], max_iter=cfg["max_iter"], threads=1)
    P.check(qo1[st1 == 0], threads=1)
    dt1 = time.perf_counter() - t1
    return dict(value=float(conv.sum() / dt), unit="converged projections/s", cores=oracle.max_threads(),
                kind="oracle",
                sample=f"{len(q)} configurations ({g_take} geodesics x {per}) of the humanoid batch, "
                       f"projection + brute-force collision check, FP64, median of {runs} runs: {dt:.2f} s",
                seconds=dt, run_seconds=times, n=int(len(q)), cpu_model=cpu_model(), nproc=os.cpu_count(),
                single_thread=dict(value=float((st1 == 0).sum() / dt1), n=int(len(q1)), seconds=dt1))


def other_workloads(M, S, FL, torch, steps):
    """The smaller configurations through the same fused path (attribution rows, not the headline):
    throughput, iteration statistics, algorithmic FLOP rate and HBM rate (inputs, outputs, status,
    iterations, residual and verdict bytes) of the whole projection step."""
    rows = {}
    for name in ("c0", "c1", "c2", "c5", "c6"):
        cfg = S.make_config(name)
        sc = cfg["scene"]
        G = M.Problem(sc.to_blob())
        if "q" in cfg:
            q = torch.from_numpy(np.ascontiguousarray(cfg["q"].T)).to("cuda", torch.float32)
        else:
            q, _, _ = build_batch(G, cfg, torch)
        n = q.shape[1]
        kw = dict(tol=cfg["tol"], max_iter=cfg["max_iter"])
        # the library's autotuner on this batch: launch shape, then (long exact-check queues) the
        # check's lane groups; the auto variant then runs what it stored
        try:
            tuned, _ = G.autotune(q, reps=3, **kw)
        except M.McError as e:
            tuned = dict(error=str(e))
        G.fallback_count(reset=True)
        out = G.project(q, **kw)
        torch.cuda.synchronize()
        fallbacks = G.fallback_count(reset=True)  # configurations continued in FP64 in one step
        ms = timed(lambda: G.project(q, out=out, **kw), steps, 2, torch)
        st = out.status.cpu().numpy()
        it = out.iters.cpu().numpy().astype(np.int64)
        vd = out.verdict.cpu().numpy()
        conv = st == 0
        byts = n * (2 * sc.d * 4 + 4 + 3)
        rows[name] = dict(configs=n, dof=sc.d, rows=sc.m, ms_per_step=ms, converged_per_s=float(conv.sum() / (ms * 1e-3)),
                          converged_frac=float(conv.mean()), iters_mean=float(it.mean()),
                          iters_p99=float(np.percentile(it, 99)),
                          collision_free_frac_of_converged=float((vd[conv] == 0).mean()) if conv.any() else None,
                          fp64_fallbacks_per_step=fallbacks, fp64_fallback_frac=fallbacks / n,
                          tflops_algorithmic=FL.batch_flops(sc, it) / (ms * 1e-3) / 1e12,
                          hbm_gbs_algorithmic=byts / (ms * 1e-3) / 1e9, tuned=tuned)
        log(f"{name}: {n} configurations, {ms:.3f} ms/step, {rows[name]['converged_per_s']:.4g} converged/s")
    return rows


def cyclic_row(G, q_in, out, kw, args, torch):
    """The cyclic mode (one step per constraint block) on the headline batch."""
    outc = G.project(q_in, variant="fused", mode="cyclic", **kw)
    ms_cyc = timed(lambda: G.project(q_in, variant="fused", mode="cyclic", out=outc, **kw), args.steps, args.warmup,
                   torch)
    st_c = outc.status.cpu().numpy()
    it_c = outc.iters.cpu().numpy().astype(np.int64)
    cyclic = dict(ms_per_step=ms_cyc, value=float((st_c == 0).sum() / (ms_cyc * 1e-3)),
                  converged_frac=float((st_c == 0).mean()), iters_mean=float(it_c.mean()),
                  iters_p99=float(np.percentile(it_c, 99)),
                  max_abs_diff_vs_stacked=float((outc.q - out.q).abs().max()))
    log(f"cyclic mode: {ms_cyc:.3f} ms/step, {cyclic['value']:.4g} converged/s, iterations {cyclic['iters_mean']:.2f}")
    return cyclic


def peak_clock_mhz():
    """The device's peak shader clock (hipDeviceAttributeClockRate = 5, in kHz), or None."""
    import ctypes
    try:
        hip = ctypes.CDLL("libamdhip64.so")
        v = ctypes.c_int(0)
        if hip.hipDeviceGetAttribute(ctypes.byref(v), 5, 0) == 0 and v.value > 0:
            return v.value / 1000.0
    except OSError:
        pass
    return None


def extend_row(M, S, G, torch, steps, shape):
    """Alg. 2 ConstrainedExtend batched (extend_batch) on the humanoid: 8,192 extensions of 8
    particles each (65,536 particle projections, as many lanes as the headline batch), then the
    interpolation and refinement levels of every surviving extension."""
    w = S.extend_workload("c3", 8192)
    raw = torch.from_numpy(np.ascontiguousarray(w["starts"].T)).to("cuda", torch.float32)
    rs = G.project(raw, tol=1e-9, max_iter=100, check=False)
    keep = (rs.status == 0).nonzero().flatten()
    qs = rs.q.index_select(1, keep).contiguous()
    qt = torch.from_numpy(np.ascontiguousarray(w["targets"].T)).to("cuda", torch.float32).index_select(1, keep)
    qt = qt.contiguous()
    eps = torch.from_numpy(w["eps"]).to("cuda", torch.float32).index_select(0, keep).contiguous()
    E = qs.shape[1]
    call = lambda: G.extend(qs, qt, eps, w["r"], w["delta"], tol=w["tol"], max_iter=w["max_iter"], **shape)
    r = call()
    ms = timed(call, steps, 1, torch, "extend")
    code = r.result.cpu().numpy()
    npts = r.n_points.cpu().numpy()
    ok = code == M.EXT_OK
    row = dict(extensions=E, particles=int(E * w["eps"].shape[1]), ms_per_call=ms,
               extensions_per_s=E / (ms * 1e-3), successful_per_s=float(ok.sum() / (ms * 1e-3)),
               codes={int(c): int((code == c).sum()) for c in np.unique(code)},
               mean_chain_points_ok=float(npts[ok].mean()) if ok.any() else None,
               r=w["r"], delta=w["delta"], n=w["n"], sigma=w["sigma"])
    log(f"extend: {E} extensions in {ms:.3f} ms ({row['extensions_per_s']:.4g}/s), codes {row['codes']}")
    return row


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-vjp", action="store_true")
    ap.add_argument("--cpu-max-configs", type=int, default=65536)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration for profiling runs)")
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true", help="use the library's default launch shape")
    ap.add_argument("--no-others", action="store_true", help="skip the C0-C2 attribution rows")
    ap.add_argument("--no-cyclic", action="store_true", help="skip the cyclic-mode row")
    ap.add_argument("--no-extend", action="store_true", help="skip the ConstrainedExtend row")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the projection shards by whole "
              "geodesics with no collective in the hot loop.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_13323_amd as M
    from paper_2604_13323_amd import flops as FL
    from paper_2604_13323_amd import scenes as S

    M.lib()  # the HIP library must be present: there is no fallback
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    torch.cuda.set_device(0)

    cfg = S.make_config("c3")
    sc = cfg["scene"]
    G = M.Problem(sc.to_blob())
    q_in, offs, _ = build_batch(G, cfg, torch)
    n = q_in.shape[1]
    tol, mi = cfg["tol"], cfg["max_iter"]
    kw = dict(tol=tol, max_iter=mi, waves_per_block=args.waves_per_block, blocks_per_cu=args.blocks_per_cu)
    out = G.project(q_in, variant="fused", **kw)
    torch.cuda.synchronize()
    log(f"humanoid batch: {n} configurations built; first projection done")
    tuning = None
    if not args.no_autotune and args.waves_per_block == 0 and args.blocks_per_cu == 0:
        from paper_2604_13323_amd import autotune
        tuning = autotune.tune(G, q_in, tol=tol, max_iter=mi)
        # the launch shape goes into the calls' options; the exact-check lane groups (where the
        # autotuner chose them) stay stored in the problem
        kw.update({k: tuning["best"][k] for k in ("waves_per_block", "blocks_per_cu", "lanes_per_config")})
        shapes = ", ".join("%dx%d: %.3f" % (r["waves_per_block"], r["blocks_per_cu"], r["ms"]) for r in tuning["table"])
        log(f"autotuned launch shape: {tuning['best']} ({shapes} ms)")

    # --- headline: fused persistent projection + collision check
    G.fallback_count(reset=True)
    ms = timed(lambda: G.project(q_in, variant="fused", out=out, **kw), args.steps, args.warmup, torch, "fused")
    status = out.status.cpu().numpy()
    iters = out.iters.cpu().numpy().astype(np.int64)
    verdict = out.verdict.cpu().numpy()
    n_conv = int((status == 0).sum())
    fallbacks = G.fallback_count(reset=True)
    value = n_conv / (ms * 1e-3)
    log(f"fused: {ms:.3f} ms/step, {value:.4g} converged projections/s, converged {n_conv}/{n}")

    # --- the dominant kernel: the persistent projection kernel of the fused step (with its broad-phase
    # walk), its launch duration from HIP events the library records around that launch alone on the
    # call's stream (queue reset, FP64 and exact-check tails excluded), one timed call after another
    G.kernel_timing(True)
    for _ in range(args.warmup):
        G.project(q_in, variant="fused", out=out, **kw)
    kms = []
    for _ in range(args.steps):
        G.project(q_in, variant="fused", out=out, **kw)
        kms.append(G.last_kernel_ms("projection"))
    G.kernel_timing(False)
    ms_kernel = float(np.mean(kms))
    ms_check = timed(lambda: G.check(out.q), args.steps, args.warmup, torch)
    # algorithmic work of one launch: the nominal per-iteration figure x the batch's Newton
    # iterations + a final residual per configuration + the broad phase the kernel runs at convergence
    flop = FL.nominal_batch_flops(sc, iters, with_broad=True)
    flop_model = FL.batch_flops(sc, iters, with_broad=True)
    achieved_tflops = flop / (ms_kernel * 1e-3) / 1e12
    log(f"persistent kernel: {ms_kernel:.4f} ms per launch (min {min(kms):.4f}), {achieved_tflops:.2f} TFLOP/s "
        f"algorithmic = {achieved_tflops / PEAK_FP32_TFLOPS:.3f} of {PEAK_FP32_TFLOPS}; check_batch alone {ms_check:.3f} ms")

    # --- the paper's composition rule: cyclic steps over the constraint blocks (same batch)
    cyclic = None
    if not args.no_cyclic:
        cyclic = cyclic_row(G, q_in, out, kw, args, torch)

    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic_projection_humanoid36.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            t = json.load(f)
        if t.get("source_hash") == source_hash():
            traffic = t.get("bytes_per_launch")

    # --- plain per-geodesic launches on the same batch
    plain = None
    if not args.no_plain:
        offs_host = np.asarray(cfg["geo_offsets"], np.int32)
        outp = G.project(q_in, variant="plain", geo_offsets=offs_host, **kw)
        ms_plain = timed(lambda: G.project(q_in, variant="plain", geo_offsets=offs_host, out=outp, **kw),
                         args.plain_steps, 1, torch)
        same = bool(torch.equal(outp.q, out.q) and torch.equal(outp.status, out.status))
        plain = dict(ms_per_step=ms_plain, value=n_conv / (ms_plain * 1e-3), launches=len(offs_host) - 1,
                     identical_outputs=same)
        log(f"plain: {ms_plain:.3f} ms/step ({plain['value']:.4g}/s), outputs identical to fused: {same}")
        # the same per-geodesic launches captured once in a HIP graph and replayed (launch cost removed)
        offs_d = torch.from_numpy(offs_host).cuda()
        outg = M.ProjectResult(q=torch.empty_like(out.q), status=torch.empty_like(out.status),
                               iters=torch.empty_like(out.iters), resid=torch.empty_like(out.resid),
                               verdict=torch.empty_like(out.verdict), geo_ok=None)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            G.project(q_in, variant="plain", geo_offsets=offs_d, geo_offsets_host=offs_host, out=outg, **kw)
        ms_pg = timed(graph.replay, args.plain_steps, 1, torch)
        same_g = bool(torch.equal(outg.q, out.q) and torch.equal(outg.status, out.status))
        plain["graph"] = dict(ms_per_step=ms_pg, value=n_conv / (ms_pg * 1e-3), identical_outputs=same_g)
        log(f"plain + hipGraph: {ms_pg:.3f} ms/step ({n_conv / (ms_pg * 1e-3):.4g}/s), identical: {same_g}")

    # --- fwd + VJP on the differentiation batch
    fv = None
    if not args.no_vjp:
        cfg4 = S.make_config("c4")
        q4, offs4, _ = build_batch(G, cfg4, torch)
        n4 = q4.shape[1]
        # the launch shape is left to the library here: this batch is larger than the lanes of the
        # one-wave launch, so it runs in the two-wave build
        kw4 = dict(kw, waves_per_block=0, blocks_per_cu=0)
        o4 = G.project(q4, variant="fused", **kw4)

        def fwd_vjp():
            G.project(q4, variant="fused", out=o4, **kw4)
            g, _ = G.path_length_grad(o4.q, offs4)
            G.vjp(o4.q, o4.status, g)

        ms4 = timed(fwd_vjp, args.steps, args.warmup, torch, "fwd_vjp")
        # the VJP kernel alone (HIP events around its launch); ~14 kFLOP per converged configuration
        # (one Newton iteration's work plus J g, the nominal per-unit VJP figure)
        g4, _ = G.path_length_grad(o4.q, offs4)
        G.kernel_timing(True)
        vms = []
        for _ in range(args.steps):
            G.vjp(o4.q, o4.status, g4)
            vms.append(G.last_kernel_ms("vjp"))
        G.kernel_timing(False)
        n4c = int((o4.status == 0).sum().item())
        vjp_tflops = 14000.0 * n4c / (np.mean(vms) * 1e-3) / 1e12
        fv = dict(value=n4 / (ms4 * 1e-3), unit="configurations/s", ms_per_step=ms4, configs=n4,
                  geodesics=len(cfg4["geo_offsets"]) - 1, vjp_kernel_ms=float(np.mean(vms)),
                  vjp_kernel_tflops=vjp_tflops, vjp_kernel_frac=vjp_tflops / PEAK_FP32_TFLOPS)
        log(f"fwd+vjp: {ms4:.3f} ms/step, {fv['value']:.4g} configurations/s; VJP kernel {np.mean(vms):.4f} ms, "
            f"{vjp_tflops:.2f} TFLOP/s")

        # the exact VJP of the map at the (off-manifold) interpolants: reverse mode through the steps
        def fwd_vjp_exact():
            G.project(q4, variant="fused", out=o4, **kw4)
            g, _ = G.path_length_grad(o4.q, offs4)
            G.vjp_exact(q4, o4.status, o4.iters, g)

        ms4x = timed(fwd_vjp_exact, max(3, args.steps // 2), 1, torch, "fwd_vjp_exact")
        G.kernel_timing(True)
        xms = []
        for _ in range(3):
            G.vjp_exact(q4, o4.status, o4.iters, g4)
            xms.append(G.last_kernel_ms("vjp"))
        G.kernel_timing(False)
        fv["exact"] = dict(value=n4 / (ms4x * 1e-3), ms_per_step=ms4x, vjp_exact_kernel_ms=float(np.mean(xms)))
        log(f"fwd+exact vjp: {ms4x:.3f} ms/step, {fv['exact']['value']:.4g} configurations/s; "
            f"exact VJP kernel {np.mean(xms):.3f} ms")

    if args.copy_calibration:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    ext = None if args.no_extend else extend_row(M, S, G, torch, min(args.steps, 10),
                                                 {k: kw[k] for k in ("waves_per_block", "blocks_per_cu")})
    others = None if args.no_others else other_workloads(M, S, FL, torch, args.steps)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(cfg, args.cpu_max_configs)
        log(f"cpu baseline: {cpu['value']:.4g} converged projections/s on {cpu['cores']} threads")

    result = {
        "metric": "converged projections/s at 36-DoF + fwd+VJP/s, fused-batched vs plain, tol 1e-6",
        "value": value,
        "unit": "converged projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "humanoid36: 65,536 configurations (2,048 geodesics x 32 interior points between "
                               "projected endpoints), 36 DoF, 20 rows, 248 robot spheres vs 500 obstacle spheres, "
                               "tol 1e-6, max 40 steps, fused persistent kernel + collision check",
                   "configs": n, "geodesics": len(cfg["geo_offsets"]) - 1},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "kernel": "k_project_persistent<humanoid36, FP32 mode>", "kernel_ms": ms_kernel,
                     "kernel_ms_min": min(kms), "flop_per_launch": flop,
                     "flop_per_launch_structural_model": flop_model,
                     "frac_vs_nonpacked_peak": achieved_tflops / PEAK_NONPACKED_TFLOPS,
                     "nonpacked_peak": PEAK_NONPACKED_TFLOPS},
        "cpu_baseline": cpu,
        "plain": plain,
        "fused_vs_plain": (value / plain["value"]) if plain else None,
        "fwd_vjp": fv,
        "cyclic_mode": cyclic,
        "extend": ext,
        "other_workloads": others,
        "stats": {"converged_frac": n_conv / n, "iters_mean": float(iters.mean()),
                  "iters_p99": float(np.percentile(iters, 99)), "iters_max": int(iters.max()),
                  "collision_free_frac_of_converged": float((verdict[status == 0] == 0).mean()) if n_conv else None,
                  "fp64_fallbacks_per_step": fallbacks / max(1, args.steps + args.warmup),
                  "check_batch_ms": ms_check, "persistent_kernel_ms": ms_kernel,
                  "launch_shape": {k: kw[k] for k in ("waves_per_block", "blocks_per_cu")},
                  "median_ms_per_step": dict(STEP_MEDIANS),
                  "cus": torch.cuda.get_device_properties(0).multi_processor_count,
                  "peak_clock_mhz": peak_clock_mhz(),
                  "autotune": tuning["table"] if tuning else None,
                  "gpu": torch.cuda.get_device_name(0)},
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
