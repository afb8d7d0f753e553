"""Launch-shape autotuner for the fused projection.

The persistent kernel's shape has two knobs: wavefronts per workgroup (1, 2, 4: how many waves
share a workgroup's LDS tile and its slice of the work queue) and resident workgroups per CU (0
= the occupancy limit). The best pair depends on the family (register and LDS footprint), the
precision mode and the batch size. `tune` times every candidate on a real batch with HIP events,
checks that all candidates give identical outputs (the launch shape must not change results),
and records the fastest per (family, dof, dtype, batch-size bucket) in a JSON cache, which
`tuned` reads back.
"""
from __future__ import annotations

import json
import os

import torch

CANDIDATES = ((1, 0), (2, 0), (4, 0), (1, 1), (1, 2), (2, 1), (4, 1))
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mcproj", "autotune.json")


def _key(G, q: torch.Tensor) -> str:
    n = q.shape[1]
    bucket = 1 << max(0, (n - 1).bit_length())  # next power of two
    return f"family{G.family}-d{G.d}-{str(q.dtype).replace('torch.', '')}-n{bucket}"


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(G, q: torch.Tensor, reps: int = 5, cache_path: str | None = DEFAULT_CACHE, **kw) -> dict:
    """Time the candidates on batch q (project kwargs in kw) and cache the fastest launch shape."""
    ref = G.project(q, variant="fused", **kw)
    table = []
    for w, b in CANDIDATES:
        out = G.project(q, variant="fused", waves_per_block=w, blocks_per_cu=b, **kw)
        torch.cuda.synchronize()
        same = bool(torch.equal(out.q, ref.q) and torch.equal(out.status, ref.status) and
                    (out.verdict is None or torch.equal(out.verdict, ref.verdict)))
        if not same:
            raise RuntimeError(f"launch shape ({w}, {b}) changed the results")
        ms = _time(lambda: G.project(q, variant="fused", waves_per_block=w, blocks_per_cu=b, out=out, **kw), reps)
        table.append(dict(waves_per_block=w, blocks_per_cu=b, ms=ms))
    best = min(table, key=lambda r: r["ms"])
    res = dict(key=_key(G, q), best=dict(waves_per_block=best["waves_per_block"], blocks_per_cu=best["blocks_per_cu"]),
               table=table)
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            try:
                with open(cache_path) as f:
                    cache = json.load(f)
            except (OSError, ValueError):
                cache = {}
        cache[res["key"]] = res["best"]
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return res


def tuned(G, q: torch.Tensor, cache_path: str = DEFAULT_CACHE) -> dict:
    """The cached launch shape for this problem and batch size, or {} (library defaults)."""
    if not os.path.exists(cache_path):
        return {}
    try:
        with open(cache_path) as f:
            return dict(json.load(f).get(_key(G, q), {}))
    except (OSError, ValueError):
        return {}
