"""Autotuner of the index's runtime knobs.

None of the knobs changes any result (every query is exact); they only
change speed. The tuner builds the index on a sample of the caller's points
and times build, kNN and range count with HIP events, in stages:

1. structure: leaf size phi, node fan-out B and the kNN traversal (seeded
   fixed-order walk, or nearest-child-first);
2. the seeded walk's knobs on the best structure (when it uses that walk and
   k <= 16): seed leaves around the query's own leaf, and the length of the
   candidate-leaf list collected before a scan (psi_set_tuning);
3. query ordering: the top curve-key bits query and box batches are sorted
   on, or input order;
4. the build's sort: the two-level bucket sort or plain LSD radix passes.

Every candidate's answers are checked to be identical to the first one's.
The cheapest candidate of each stage (by a weighted sum of the times) is
kept; all candidates with their times are returned and cached in a JSON
file keyed by (GPU architecture, dim, curve, size bucket, k).

Kernel tile shapes (the sort's tile of pairs, its digit width, the bucket
count) are compile-time constants sized to the LDS budgets of their
kernels; they are not searched here.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

from . import (FLAG_INPUT_ORDER, FLAG_KNN_NEAREST_FIRST, FLAG_SORT_BUCKETS, FLAG_SORT_LSD, Index, psi_set_tuning,
               to_u32, to_u64)

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "psi_autotune.json")

LEAF_SIZES = (16, 24, 32)
FANOUTS = (4, 8, 16, 32)
VARIANTS = (0, FLAG_KNN_NEAREST_FIRST)
SEED_LEAVES = (1, 3, 5, 7)
CAND_LENGTHS = (8, 16, 32)
ORDER_BITS = (16, 24, 32)
DEFAULT_TUNING = {"knn_seed_leaves": 3, "knn_cand": 16, "order_bits": 24}


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
         candidates=None, cache_path: str | None = DEFAULT_CACHE, use_cache: bool = True,
         stages: bool = True) -> dict:
    """Pick (leaf_size, fanout, flags, tuning) for this kind of data; returns a
    dict with the choice and the measured times of every candidate.
    `candidates` (leaf size, fan-out, flags) replaces stage 1's grid;
    stages=False stops after stage 1."""
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
    ref = [None]

    def run(stage, phi, fan, flags, tuning, do_build=True, do_knn=True, do_range=True):
        ix = Index(dim, curve, phi, fan, device=dev, stream=stream, flags=flags)
        psi_set_tuning(ix._h, **tuning)
        t_build = _time(lambda: ix.build(d_pts), stream) if do_build else None
        if not do_build:
            ix.build(d_pts)
        out = {}

        def knn():
            out["knn"] = ix.knn(d_q, k)

        def rc():
            out["rc"] = ix.range_count(d_b)

        t_knn = _time(knn, stream) if do_knn else None
        t_range = _time(rc, stream) if (do_range and d_b is not None) else None
        if "knn" not in out:
            knn()
        if d_b is not None and "rc" not in out:
            rc()
        ix.sync()
        got = (to_u32(out["knn"][0]), to_u64(out["knn"][1]), to_u64(out["rc"]) if d_b is not None else None)
        if ref[0] is None:
            ref[0] = got
        else:  # the knobs must not change any answer
            for a, b in zip(ref[0], got):
                if a is not None and not np.array_equal(a, b):
                    raise RuntimeError(f"candidate {(phi, fan, flags, tuning)} changed a query result")
        ix.close()
        cost = (weights[0] * (t_build or 0.0) + weights[1] * (t_knn or 0.0) + weights[2] * (t_range or 0.0))
        return dict(stage=stage, leaf_size=phi, fanout=fan, flags=flags, tuning=dict(tuning), build_ms=t_build,
                    knn_ms=t_knn, range_ms=t_range, cost=cost)

    results = [run("structure", phi, fan, flags, DEFAULT_TUNING) for phi, fan, flags in candidates]
    best = min(results, key=lambda r: r["cost"])
    phi, fan, flags, tuning = best["leaf_size"], best["fanout"], best["flags"], dict(DEFAULT_TUNING)
    if stages:
        if k <= 16 and not (flags & FLAG_KNN_NEAREST_FIRST):
            walk = [run("knn_walk", phi, fan, flags, dict(tuning, knn_seed_leaves=s, knn_cand=c),
                        do_build=False, do_range=False)
                    for s, c in itertools.product(SEED_LEAVES, CAND_LENGTHS)]
            w = min(walk, key=lambda r: r["knn_ms"])
            tuning = dict(w["tuning"])
            results += walk
        order = [run("order", phi, fan, flags & ~FLAG_INPUT_ORDER, dict(tuning, order_bits=b), do_build=False)
                 for b in ORDER_BITS]
        order.append(run("order", phi, fan, flags | FLAG_INPUT_ORDER, tuning, do_build=False))
        o = min(order, key=lambda r: r["cost"])
        flags, tuning = o["flags"], dict(o["tuning"])
        results += order
        base = flags & ~(FLAG_SORT_BUCKETS | FLAG_SORT_LSD)
        sort = [run("build_sort", phi, fan, base | f, tuning, do_knn=False, do_range=False)
                for f in (0, FLAG_SORT_BUCKETS, FLAG_SORT_LSD)]
        s = min(sort, key=lambda r: r["build_ms"])
        flags = s["flags"]
        results += sort
    choice = dict(key=key, leaf_size=phi, fanout=fan, flags=flags, tuning=tuning, sample_n=n, candidates=results)
    if cache_path:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            data = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
            data[key] = choice
            json.dump(data, open(cache_path, "w"), indent=1)
        except (OSError, ValueError):
            pass
    return dict(choice, cached=False)


def apply(index, choice: dict):
    """Set a tuned choice's runtime knobs on an index built with its leaf
    size, fan-out and flags."""
    psi_set_tuning(index._h, **choice.get("tuning", DEFAULT_TUNING))
