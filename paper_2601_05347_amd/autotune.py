"""Autotuner of the index's runtime knobs.

Knobs: leaf size phi, node fan-out B, the kNN traversal variant (seeded
fixed-order walk, or nearest-child-first) and whether query batches are
processed in curve order. None of them changes any result (every query is
exact); they only change speed. The tuner builds the index on a sample of
the caller's points, times build, kNN and range count with HIP events for
every candidate, checks that all candidates return identical answers, and
keeps the cheapest by a weighted sum of the three times. Choices are cached
in a JSON file keyed by (GPU architecture, dim, curve, size bucket, k).
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

from . import FLAG_INPUT_ORDER, FLAG_KNN_NEAREST_FIRST, Index, to_u32, to_u64

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "psi_autotune.json")

LEAF_SIZES = (16, 24, 32)
FANOUTS = (4, 8, 16, 32)
VARIANTS = (0, FLAG_KNN_NEAREST_FIRST)


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def cache_key(dim: int, curve: int, n: int, k: int) -> str:
    bucket = int(round(math.log10(max(n, 1))))
    return f"{_arch()}|{dim}d|curve{curve}|n1e{bucket}|k{k}"


def _time(fn, stream, reps: int = 3) -> float:
    import torch
    fn()  # warm: sizes buffers
    stream.synchronize()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def tune(dim: int, curve: int, pts, queries, k: int = 10, boxes=None, weights=(1.0, 1.0, 1.0),
         candidates=None, cache_path: str | None = DEFAULT_CACHE, use_cache: bool = True) -> dict:
    """Pick (leaf_size, fanout, flags) for this kind of data; returns a dict
    with the choice and the measured times of every candidate."""
    import torch
    n = len(pts)
    key = cache_key(dim, curve, n, k)
    if use_cache and cache_path and os.path.exists(cache_path):
        try:
            cached = json.load(open(cache_path)).get(key)
            if cached:
                return dict(cached, cached=True)
        except (OSError, ValueError):
            pass
    if candidates is None:
        candidates = [(phi, b, v) for phi, b, v in itertools.product(LEAF_SIZES, FANOUTS, VARIANTS)]
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream(dev)
    d_pts = torch.from_numpy(np.ascontiguousarray(pts, np.uint32).view(np.int32)).to(dev)
    d_q = torch.from_numpy(np.ascontiguousarray(queries, np.uint32).view(np.int32)).to(dev)
    d_b = (torch.from_numpy(np.ascontiguousarray(boxes, np.uint32).view(np.int32)).to(dev)
           if boxes is not None else None)
    results, ref = [], None
    for phi, fan, flags in candidates:
        ix = Index(dim, curve, phi, fan, device=dev, stream=stream, flags=flags)
        t_build = _time(lambda: ix.build(d_pts), stream)
        out = {}

        def knn():
            out["knn"] = ix.knn(d_q, k)

        t_knn = _time(knn, stream)
        t_range = 0.0
        if d_b is not None:
            def rc():
                out["rc"] = ix.range_count(d_b)
            t_range = _time(rc, stream)
        ix.sync()
        got = (to_u32(out["knn"][0]), to_u64(out["knn"][1]), to_u64(out["rc"]) if d_b is not None else None)
        if ref is None:
            ref = got
        else:  # the knobs must not change any answer
            for a, b in zip(ref, got):
                if a is not None and not np.array_equal(a, b):
                    raise RuntimeError(f"candidate {(phi, fan, flags)} changed a query result")
        cost = weights[0] * t_build + weights[1] * t_knn + weights[2] * t_range
        results.append(dict(leaf_size=phi, fanout=fan, flags=flags, build_ms=t_build, knn_ms=t_knn,
                            range_ms=t_range, cost=cost))
        ix.close()
    best = min(results, key=lambda r: r["cost"])
    choice = dict(key=key, leaf_size=best["leaf_size"], fanout=best["fanout"], flags=best["flags"],
                  sample_n=n, candidates=results)
    if cache_path:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            data = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
            data[key] = choice
            json.dump(data, open(cache_path, "w"), indent=1)
        except (OSError, ValueError):
            pass
    return dict(choice, cached=False)
