#!/usr/bin/env python3
"""Benchmark of the SPaC-tree hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input:
  build(n) -> batch_insert(m) -> batch_delete(m existing ids)
  -> kNN(nq queries, k) -> range_count(nb boxes) -> range_report(nb boxes).
Default workload: 3D SPaC-H (Hilbert), n = 1e8 points with 21-bit coordinates
(uniform), m = 1e6, 1e7 kNN queries with k = 10, 1e6 boxes with sides
log-uniform in 2^8..2^18. Inputs are resident in HBM before timing starts.

`value` is the build & batch-update throughput in Mpoints/s:
(n + m + m) / (t_build + t_insert + t_delete). kNN queries/s and range
boxes/s of the same steps are reported under `phases`.

Prints ONE JSON line. `--gpus N` with N > 1 is refused: the library runs on
one GPU (the sharded design is described but not built).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpoints/s build & batch-update, kNN queries/s (1e8 pts, 3D); p99 latency"
HBM_PEAK_GBS = 8000.0
CALIB_BYTES = 1 << 30

WORKLOADS = {
    # the metric's configuration: 3D, 1e8 points, 21-bit coordinates
    "3d-1e8": dict(dim=3, bits=21, n=100_000_000, m=1_000_000, nq=10_000_000, k=10, nb=1_000_000),
    # 2D, 1e8 points in [0, 2^30)^2
    "2d-1e8": dict(dim=2, bits=30, n=100_000_000, m=1_000_000, nq=10_000_000, k=10, nb=1_000_000),
    # small configuration (seconds on the oracle)
    "2d-1e6": dict(dim=2, bits=30, n=1_000_000, m=100_000, nq=10_000, k=10, nb=10_000),
    # serving: resident 3D SPaC-H of 5e7 points, mixed Poisson request stream
    "serve": dict(dim=3, bits=21, n=50_000_000, m=0, nq=0, k=10, nb=0),
    # 4096 independent 2D SPaC-Z indexes (sizes log-uniform 1e3..1e6), kNN k = 8
    "multi": dict(dim=2, bits=30, n=0, m=0, nq=0, k=8, nb=0),
    # P-Orth tree (Sec. 3) beside the SPaC-H tree on the 3d-1e8 inputs: build,
    # insert 1e6, delete 1e6, 1e7 10-NN queries, 1e6 range counts and reports
    "orth": dict(dim=3, bits=21, n=100_000_000, m=1_000_000, nq=10_000_000, k=10, nb=1_000_000),
    # the SPaC tree in the paper's shape beside the directory SPaC-H tree (3D)
    "bst": dict(dim=3, bits=21, n=100_000_000, m=1_000_000, nq=10_000_000, k=10, nb=1_000_000),
    # the same in 2D, coordinates in [0, 2^30)^2
    "orth2d": dict(dim=2, bits=30, n=100_000_000, m=1_000_000, nq=10_000_000, k=10, nb=1_000_000),
    # incremental workload: 3D, 1e8 points inserted into an empty index in n/b
    # batches, then deleted in n/b batches; 1e7 10-NN queries at the halfway points
    "incr": dict(dim=3, bits=21, n=100_000_000, m=0, nq=10_000_000, k=10, nb=0),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="3d-1e8", choices=sorted(WORKLOADS))
    ap.add_argument("--dist", default="uniform", choices=["uniform", "varden", "sweepline"])
    ap.add_argument("--curve", default="hilbert", choices=["hilbert", "morton"])
    ap.add_argument("--leaf", type=int, default=32)
    ap.add_argument("--fanout", type=int, default=8)
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--ops", default="build,insert,delete,knn,range")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-sample", type=int, default=32_000_000, help="points in the oracle's timed sample")
    ap.add_argument("--cpu-queries", type=int, default=512, help="queries and boxes in the oracle's timed sample")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving block of the default line")
    ap.add_argument("--serve-requests", type=int, default=600, help="requests in the default line's serving block")
    ap.add_argument("--requests", type=int, default=4000, help="serve: requests per stream")
    ap.add_argument("--rho", default="0.5,0.8,1.2", help="serve: loads relative to the plain path's capacity")
    ap.add_argument("--serve-paths", default="plain,batched,library", help="serve: the paths to run")
    ap.add_argument("--indexes", type=int, default=4096, help="multi: number of indexes")
    ap.add_argument("--batch-frac", default="0.1,0.01,0.001,0.0001", help="incr: batch sizes as fractions of n")
    ap.add_argument("--tree", default="spac", choices=["spac", "orth"],
                    help="incr: the SPaC tree (curve from --curve) or the P-Orth tree")
    ap.add_argument("--sorted-leaves", action="store_true",
                    help="keep every leaf in (key, id) order after updates (the total-order ablation)")
    return ap.parse_args()


# The source files whose code decides each kernel family's memory traffic
# (its own file and the device helpers it includes).
FAMILY_SOURCES = {
    "radix_first": ["k_sort.hip"], "radix_pass": ["k_sort.hip"], "encode_hist": ["k_sort.hip"],
    "local_sort": ["k_bucket.hip"], "local_sort_wide": ["k_bucket.hip"], "local_sort_huge": ["k_bucket.hip"],
    "bucket_starts": ["k_bucket.hip"],
    "radix_big": ["k_bucket.hip"], "leaf_fill": ["k_build.hip"], "nodes": ["k_build.hip"],
    "knn": ["k_query.hip"], "range_count": ["k_query.hip"], "range_report": ["k_query.hip"],
}
DEVICE_HELPERS = ["psi_dev.h", "psi_hilbert.h"]


def src_hash(family: str) -> str:
    """SHA-256 over the sources of a kernel family, with comments and blank
    space left out: counters taken on the code stay valid across comment
    edits and across changes to other kernels."""
    import hashlib
    import re
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2601_05347_amd", "csrc")
    for f in FAMILY_SOURCES[family] + DEVICE_HELPERS:
        code = open(os.path.join(d, f)).read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(f.encode())
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def profiled_traffic(profile: str, family: str):
    """HBM bytes per launch of a kernel family recorded by rocprofv3 counter
    runs, if none of its sources changed since (the profile carries their
    hash on the family's line: `traffic[family]: bytes sha256`)."""
    import re
    try:
        txt = open(os.path.join(ROOT, "profiles", profile)).read()
    except OSError:
        return None
    m = re.search(r"traffic\[%s\]:\s*(\d+)\s+([0-9a-f]{64})" % re.escape(family), txt)
    if not m or family not in FAMILY_SOURCES or m.group(2) != src_hash(family):
        return None
    return int(m.group(1))


CPU_THREADS = 16  # the host cores one GPU's box share has


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, args, full=None):
    """The oracle timed on bounded samples of the same workload: build and
    updates on one core over a sample of the points, then (given the full
    point set, its queries and boxes) brute-force kNN and range counts over
    all n points for a seeded sample of queries and boxes on CPU_THREADS
    threads, reported per query (no extrapolation in n)."""
    import numpy as np

    import oracle
    import synth
    dim, bits = cfg["dim"], cfg["bits"]
    n = min(args.cpu_sample, cfg["n"])
    m = max(1, n // 100)
    data, ins, _ = synth.workload(args.dist, dim, bits, args.seed, n=n, n_insert=m, n_query=0)
    dels = synth.delete_ids(np.arange(n + m, dtype=np.uint32), m, args.seed)
    ref = oracle.RefIndex(dim, 1 if args.curve == "hilbert" else 0, args.leaf, args.fanout)
    t0 = time.perf_counter()
    ref.build(data)
    ref.batch_insert(ins)
    ref.batch_delete(dels)
    dt = time.perf_counter() - t0
    del ref, data, ins, dels
    out = {"value": round((n + 2 * m) / dt / 1e6, 3), "unit": "Mpoints/s", "cores": 1, "kind": "oracle",
           "sample": f"build {n} + insert {m} + delete {m} {dim}D {args.dist} {args.curve} points, "
                     f"single-threaded std::sort/std::merge oracle, {dt:.2f} s",
           "host_cores": os.cpu_count(), "cpu_model": cpu_model()}
    if full is not None:
        pts, q, boxes, k = full
        rows = synth.sample_rows(len(q), args.cpu_queries, args.seed + 11)
        t0 = time.perf_counter()
        oracle.knn_points(pts, q[rows], k, threads=CPU_THREADS)
        tk = time.perf_counter() - t0
        brows = synth.sample_rows(len(boxes), args.cpu_queries, args.seed + 12)
        t0 = time.perf_counter()
        oracle.range_count_points(pts, boxes[brows], threads=CPU_THREADS)
        tr = time.perf_counter() - t0
        out["knn"] = {"value": round(len(rows) / tk, 3), "unit": "queries/s", "cores": CPU_THREADS,
                      "ms_per_query": round(tk * 1e3 / len(rows), 3),
                      "sample": f"{len(rows)} seeded {k}-NN queries, brute force over all {len(pts)} points, "
                                f"{tk:.2f} s"}
        out["range_count"] = {"value": round(len(brows) / tr, 3), "unit": "boxes/s", "cores": CPU_THREADS,
                              "ms_per_box": round(tr * 1e3 / len(brows), 3),
                              "sample": f"{len(brows)} seeded boxes, scan of all {len(pts)} points, {tr:.2f} s"}
    return out


def serve_runs(n0, n_requests, rhos, seed, leaf, fanout, paths=("plain", "batched", "library"), probe_n=400):
    """Serving: a resident 3D SPaC-H index of n0 uniform points and a Poisson
    stream of mixed requests at rho times the plain path's capacity, served
    by each path on a fresh index; p50/p99 per request type and throughput."""
    import numpy as np
    import torch

    import paper_2601_05347_amd as psi
    import synth
    from paper_2601_05347_amd import serve
    cfg = WORKLOADS["serve"]
    dim, bits = cfg["dim"], cfg["bits"]
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    base = synth.uniform(n0, dim, bits, seed)
    reqs = synth.request_stream(n_requests, n0, dim, bits, seed + 7, rate_per_s=1.0)
    log(f"serve: {len(reqs)} requests generated in {time.perf_counter() - t:.1f} s")
    d_base = torch.from_numpy(base.view(np.int32)).to(dev)

    def fresh():
        ix = psi.Index(dim, psi.HILBERT, leaf, fanout, device=dev)
        psi.psi_build(ix._h, d_base, n0)
        ix.sync()
        return ix

    # capacity of the plain path: back-to-back service of a prefix of the stream
    probe = [dict(r) for r in reqs[:probe_n]]
    ix = fresh()
    serve.PlainServer(ix).run(probe, realtime=False)
    lam_plain = len(probe) / probe[-1]["done_s"]  # back-to-back service from t = 0
    log(f"serve: plain path capacity {lam_plain:.1f} requests/s")
    ix.close()
    classes = {"plain": serve.PlainServer, "batched": serve.BatchServer, "library": serve.DeviceServer}
    runs = {}
    for rho in rhos:
        lam = rho * lam_plain
        stream_r = [dict(r, arrival=r["arrival"] / lam) for r in reqs]
        res = {}
        for name in paths:
            ix = fresh()
            rs = [dict(r) for r in stream_r]
            if name == "library":
                classes[name](ix).run(rs, realtime=True, n_live=n0, bits=bits)
            else:
                classes[name](ix).run(rs, realtime=True)
            ix.sync()
            res[name] = serve.summarize(rs)
            log(f"serve rho={rho} {name}: p50 {res[name]['all']['p50_ms']:.1f} ms, p99 {res[name]['all']['p99_ms']:.1f} "
                f"ms, {res[name]['throughput_req_s']:.1f} req/s")
            ix.close()
            del rs
        runs[f"rho={rho}"] = res
    return lam_plain, runs


def bench_serve(args):
    """Serving configuration: plain per-request path vs continuous batching
    (the Python scheduler and the library's server)."""
    cfg = WORKLOADS["serve"]
    n0 = args.n or cfg["n"]
    paths = tuple(args.serve_paths.split(","))
    lam_plain, runs = serve_runs(n0, args.requests, [float(x) for x in args.rho.split(",")], args.seed, args.leaf,
                                 args.fanout, paths=paths)
    b = runs[max(runs)][paths[-1]]
    out = {"metric": "p99 latency (ms) of mixed requests, continuous batching, 1 GPU", "value": round(b["all"]["p99_ms"], 3),
           "unit": "ms", "n_gpus": 1, "steps": args.requests, "warmup": 0, "ms_per_step": None,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u32/u64",
           "data": "synthetic",
           "config": {"workload": "serve: resident 3D SPaC-H, uniform, library server", "n0": n0,
                      "requests": args.requests, "mix": "40/20/30/10 insert/delete/knn/range",
                      "plain_capacity_req_s": round(lam_plain, 2)},
           "runs": runs}
    print(json.dumps(out), flush=True)


def bench_incr(args):
    """The paper's incremental workload (Sec. 5.1): build from empty by n/b
    batch insertions, empty by n/b batch deletions (ids in insertion order),
    10-NN queries in and out of distribution after half of each, beside the
    same queries on static builds of the same points. Every batch call is
    timed; the queries are not part of the update totals."""
    import numpy as np
    import torch

    import paper_2601_05347_amd as psi
    import synth
    cfg = WORKLOADS["incr"]
    dim, bits, k = cfg["dim"], cfg["bits"], args.k or cfg["k"]
    n = args.n or cfg["n"]
    nq = cfg["nq"] if n >= 10_000_000 else max(1000, n // 10)
    curve = psi.HILBERT if args.curve == "hilbert" else psi.MORTON
    dist = args.dist
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    t = time.perf_counter()
    data = synth.points(dist, n, dim, bits, args.seed)
    ind = synth.points("uniform" if dist == "sweepline" else dist, nq, dim, bits, args.seed + 3, synth.P_QUERY)
    ood = synth.points("uniform" if dist == "varden" else "varden", nq, dim, bits, args.seed + 4, synth.P_QUERY)
    log(f"incr: {n} {dist} points, 2 x {nq} queries generated in {time.perf_counter() - t:.1f} s")
    d_data = torch.from_numpy(data.view(np.int32)).to(dev)
    d_q = {"ind": torch.from_numpy(ind.view(np.int32)).to(dev), "ood": torch.from_numpy(ood.view(np.int32)).to(dev)}
    d_ids = torch.arange(n, dtype=torch.int32, device=dev)
    half = n // 2
    orth = args.tree == "orth"
    if orth:
        new_tree = lambda flags=0: psi.Orth(dim, args.leaf, device=dev)  # noqa: E731
        build, insert, delete, knn = (psi.psi_orth_build, psi.psi_orth_batch_insert, psi.psi_orth_batch_delete,
                                      psi.psi_orth_knn)
    else:
        new_tree = lambda flags=0: psi.Index(dim, curve, args.leaf, args.fanout, device=dev, flags=flags)  # noqa: E731
        build, insert, delete, knn = psi.psi_build, psi.psi_batch_insert, psi.psi_batch_delete, psi.psi_knn

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def queries(ix):
        out, ms = {}, {}
        for name, q in d_q.items():
            ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
            d2 = torch.empty((nq, k), dtype=torch.int64, device=dev)
            a = ev()
            knn(ix._h, q, nq, k, ids, d2)
            b = ev()
            b.synchronize()
            out[name], ms[name] = (ids, d2), round(a.elapsed_time(b), 3)
        return out, ms

    # static references: the first half (ids 0 .. n/2 - 1) and the second half
    # (built alone its ids are 0 .. n/2 - 1: the incremental ids minus n/2)
    st1 = new_tree()
    build(st1._h, d_data[:half], half)
    ref1, ms1 = queries(st1)
    del st1
    st2 = new_tree()
    build(st2._h, d_data[half:], n - half)
    ref2, ms2 = queries(st2)
    del st2
    runs = {}
    for frac in [float(x) for x in args.batch_frac.split(",")]:
        s = max(1, int(round(n * frac)))
        nbat = n // s
        ix = new_tree(psi.FLAG_SORTED_LEAVES if args.sorted_leaves else 0)
        build(ix._h, d_data[:0], 0)
        torch.cuda.synchronize()
        ins_ms = del_ms = 0.0
        same = True
        a = ev()
        for i in range(nbat):
            insert(ix._h, d_data[i * s:(i + 1) * s], s, None)
            if i == nbat // 2 - 1:
                b = ev()
                b.synchronize()
                ins_ms += a.elapsed_time(b)
                got, q_ins = queries(ix)
                if (i + 1) * s == half:
                    for name in got:
                        same &= bool(torch.equal(got[name][1], ref1[name][1]) and torch.equal(got[name][0], ref1[name][0]))
                a = ev()
        b = ev()
        b.synchronize()
        ins_ms += a.elapsed_time(b)
        a = ev()
        for i in range(nbat):
            delete(ix._h, d_ids[i * s:(i + 1) * s], s, None)
            if i == nbat // 2 - 1:
                b = ev()
                b.synchronize()
                del_ms += a.elapsed_time(b)
                got, q_del = queries(ix)
                if (i + 1) * s == half and nbat * s == n:
                    for name in got:
                        gi, gd = got[name]
                        ri, rd = ref2[name]
                        same &= bool(torch.equal(gd, rd) and torch.equal(gi, torch.where(ri >= 0, ri + half, ri)))
                a = ev()
        b = ev()
        b.synchronize()
        del_ms += a.elapsed_time(b)
        ix.sync()
        left = ix.size()[0] if orth else ix.size()
        del ix
        runs[f"b={frac}"] = {"batch": s, "batches": nbat, "insert_ms": round(ins_ms, 3), "delete_ms": round(del_ms, 3),
                             "insert_mpts_s": round(nbat * s / ins_ms / 1e3, 1),
                             "delete_mpts_s": round(nbat * s / del_ms / 1e3, 1),
                             "knn_ms_after_half_inserts": q_ins, "knn_ms_after_half_deletes": q_del,
                             "left_after_deletes": left, "results_identical_to_static": same}
        log(f"incr b={frac}: {nbat} x {s}: insert {ins_ms:.1f} ms, delete {del_ms:.1f} ms, "
            f"kNN after half {q_ins} / {q_del} ms, identical {same}")
    small = runs[min(runs, key=lambda r: runs[r]["batch"])]
    tot = small["insert_ms"] + small["delete_ms"]
    out = {"metric": "incremental build & empty by n/b batches: Mpoints/s (smallest b)",
           "value": round(2 * small["batches"] * small["batch"] / tot / 1e3, 2), "unit": "Mpoints/s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": round(tot, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32/u64", "data": "synthetic",
           "config": {"workload": f"incremental: {dim}D {dist} {'P-Orth' if orth else args.curve}", "n": n,
                      "queries": nq, "k": k,
                      "leaf_size": args.leaf, "fanout": args.fanout, "sorted_leaves": args.sorted_leaves},
           "static_knn_ms": {"first_half": ms1, "second_half": ms2}, "runs": runs}
    print(json.dumps(out), flush=True)


def bench_orth(args):
    """P-Orth tree (Sec. 3) and SPaC-H tree on the same inputs (those of the
    3d-1e8 workload): per step, a build of each, a batch insert and a batch
    delete, then kNN, range count and range report on each. Every phase is timed with HIP events on the
    stream; the builds include their readbacks."""
    import numpy as np
    import torch

    import paper_2601_05347_amd as psi
    import synth
    cfg = dict(WORKLOADS[args.workload])
    if args.n:
        cfg["n"] = args.n
    dim, bits, n, nq, k, nb = (cfg[x] for x in ("dim", "bits", "n", "nq", "k", "nb"))
    k = args.k or k
    nq = min(nq, max(1000, n // 10))
    nb = min(nb, max(1000, n // 100))
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    m = cfg["m"]
    data, ins, q = synth.workload(args.dist, dim, bits, args.seed, n=n, n_insert=m, n_query=nq)
    dels = synth.delete_ids(np.arange(n + m, dtype=np.uint32), m, args.seed)
    boxes = synth.boxes(q[:nb], bits, args.seed)
    log(f"orth: inputs generated in {time.perf_counter() - t:.1f} s")
    d_data = torch.from_numpy(data.view(np.int32)).to(dev)
    d_ins = torch.from_numpy(ins.view(np.int32)).to(dev)
    d_dels = torch.from_numpy(dels.view(np.int32)).to(dev)
    d_q = torch.from_numpy(q.view(np.int32)).to(dev)
    d_boxes = torch.from_numpy(boxes.view(np.int32)).to(dev)
    del data, q, ins
    stream = torch.cuda.current_stream(dev)
    trees = {"orth": psi.Orth(dim, args.leaf, device=dev, stream=stream),
             "spac_h": psi.Index(dim, psi.HILBERT, args.leaf, args.fanout, device=dev, stream=stream)}
    api = {"orth": (psi.psi_orth_build, psi.psi_orth_batch_insert, psi.psi_orth_batch_delete, psi.psi_orth_knn,
                    psi.psi_orth_range_count, psi.psi_orth_range_report),
           "spac_h": (psi.psi_build, psi.psi_batch_insert, psi.psi_batch_delete, psi.psi_knn, psi.psi_range_count,
                      psi.psi_range_report)}
    new_ids = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    nd = torch.zeros(1, dtype=torch.int64, device=dev)
    k_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    k_d2 = torch.empty((nq, k), dtype=torch.int64, device=dev)
    cnt = torch.empty(nb, dtype=torch.int64, device=dev)
    off = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
    rids, res, outs = {}, {}, {}
    for name, tr in trees.items():
        build, insert, delete, knn, rcount, rreport = api[name]
        h = tr._h
        ms = {p: [] for p in ("build", "insert", "delete", "knn", "range_count", "range_report")}
        for it in range(args.warmup + args.steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
            ev[0].record(stream)
            build(h, d_data, n)
            ev[1].record(stream)
            insert(h, d_ins, m, new_ids)
            ev[2].record(stream)
            delete(h, d_dels, m, nd)
            ev[3].record(stream)
            knn(h, d_q, nq, k, k_ids, k_d2)
            ev[4].record(stream)
            rcount(h, d_boxes, nb, cnt)
            ev[5].record(stream)
            if name not in rids:
                torch.cumsum(cnt, 0, out=off[1:])
                rids[name] = torch.empty(max(int(off[-1].item()), 1), dtype=torch.int32, device=dev)
                ev[5].record(stream)
            rreport(h, d_boxes, nb, off, rids[name])
            ev[6].record(stream)
            ev[6].synchronize()
            if it >= args.warmup:
                for j, p in enumerate(ms):
                    ms[p].append(ev[j].elapsed_time(ev[j + 1]))
        tr.sync()
        outs[name] = (k_ids.clone(), k_d2.clone(), cnt.clone())
        med = {p: round(float(np.median(v)), 3) for p, v in ms.items()}
        res[name] = {"ms": med, "build_mpts_s": round(n / med["build"] / 1e3, 1),
                     "insert_mpts_s": round(m / med["insert"] / 1e3, 1),
                     "delete_mpts_s": round(m / med["delete"] / 1e3, 1),
                     "knn_mq_s": round(nq / med["knn"] / 1e3, 1),
                     "range_count_mbox_s": round(nb / med["range_count"] / 1e3, 2),
                     "range_report_mbox_s": round(nb / med["range_report"] / 1e3, 2)}
        if name == "orth":
            nn, nl, hh = tr.shape()
            res[name]["shape"] = {"nodes": nn, "leaves": nl, "height": hh}
            tr.prof_enable(True)
            tr.prof_reset()
            build(h, d_data, n)
            insert(h, d_ins, m, new_ids)
            delete(h, d_dels, m, nd)
            knn(h, d_q, nq, k, k_ids, k_d2)
            fam = {}
            for f in ("encode_hist", "radix_first", "radix_pass", "bucket_starts", "local_sort", "local_sort_wide",
                      "local_sort_huge", "radix_big", "orth_marks", "orth_nodes", "orth_boxes", "orth_merge", "orth_knn", "order", "radix_order"):
                fms, nl_, _ = tr.prof_get(f)
                if nl_:
                    fam[f] = round(fms, 3)
            tr.prof_enable(False)
            res[name]["families_ms"] = fam
        log(f"{name}: {res[name]}")
    o, sp = res["orth"], res["spac_h"]
    a, b = outs["orth"], outs["spac_h"]
    identical = all(bool(torch.equal(x, y)) for x, y in zip(a, b))
    out = {"metric": "P-Orth build Mpoints/s (1e8 pts, 3D); updates, kNN and range beside SPaC-H", "value": o["build_mpts_s"],
           "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(sum(o["ms"].values()), 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32/u64", "data": "synthetic",
           "config": {"workload": f"orth: {dim}D {args.dist} P-Orth vs SPaC-H", "n": n, "queries": nq, "k": k,
                      "boxes": nb, "leaf_size": args.leaf},
           "orth": o, "spac_h": sp,
           "orth_over_spac_h": {p: round(sp["ms"][p] / o["ms"][p], 3) for p in o["ms"]},
           "knn_and_counts_identical": identical}
    print(json.dumps(out), flush=True)


def bench_bst(args):
    """The SPaC tree in the paper's shape (BuildSorted builds, join-based batch
    updates, leaf wrap 40) beside the SPaC-H directory tree on the same inputs
    (those of the 3d-1e8 workload): per step, a build of each, a batch insert
    and a batch delete, then kNN, range count and range report on each. Every
    phase is timed with HIP events on the stream; the paper-shape tree's
    calls include their readbacks."""
    import numpy as np
    import torch

    import paper_2601_05347_amd as psi
    import synth
    cfg = dict(WORKLOADS["3d-1e8"])
    if args.n:
        cfg["n"] = args.n
    dim, bits, n, nq, k, nb, m = (cfg[x] for x in ("dim", "bits", "n", "nq", "k", "nb", "m"))
    k = min(args.k or k, 16)
    nq = min(nq, max(1000, n // 10))
    nb = min(nb, max(1000, n // 100))
    m = min(m, max(1000, n // 100))
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    data, ins, q = synth.workload(args.dist, dim, bits, args.seed, n=n, n_insert=m, n_query=nq)
    dels = synth.delete_ids(np.arange(n + m, dtype=np.uint32), m, args.seed)
    boxes = synth.boxes(q[:nb], bits, args.seed)
    log(f"bst: inputs generated in {time.perf_counter() - t:.1f} s")
    d_data = torch.from_numpy(data.view(np.int32)).to(dev)
    d_ins = torch.from_numpy(ins.view(np.int32)).to(dev)
    d_dels = torch.from_numpy(dels.view(np.int32)).to(dev)
    d_q = torch.from_numpy(q.view(np.int32)).to(dev)
    d_boxes = torch.from_numpy(boxes.view(np.int32)).to(dev)
    del data, q, ins
    stream = torch.cuda.current_stream(dev)
    trees = {"paper_shape": psi.Bst(dim, psi.HILBERT, 40, device=dev, stream=stream),
             "spac_h": psi.Index(dim, psi.HILBERT, args.leaf, args.fanout, device=dev, stream=stream)}
    api = {"paper_shape": (psi.psi_bst_build, psi.psi_bst_batch_insert, psi.psi_bst_batch_delete, psi.psi_bst_knn,
                           psi.psi_bst_range_count, psi.psi_bst_range_report),
           "spac_h": (psi.psi_build, psi.psi_batch_insert, psi.psi_batch_delete, psi.psi_knn, psi.psi_range_count,
                      psi.psi_range_report)}
    new_ids = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    nd = torch.zeros(1, dtype=torch.int64, device=dev)
    k_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    k_d2 = torch.empty((nq, k), dtype=torch.int64, device=dev)
    cnt = torch.empty(nb, dtype=torch.int64, device=dev)
    off = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
    rids, res, outs = {}, {}, {}
    for name, tr in trees.items():
        build, insert, delete, knn, rcount, rreport = api[name]
        h = tr._h
        ms = {p: [] for p in ("build", "insert", "delete", "knn", "range_count", "range_report")}
        for it in range(args.warmup + args.steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
            log(f"bst: {name} step {it}")
            ev[0].record(stream)
            build(h, d_data, n)
            ev[1].record(stream)
            insert(h, d_ins, m, new_ids)
            ev[2].record(stream)
            delete(h, d_dels, m, nd)
            ev[3].record(stream)
            knn(h, d_q, nq, k, k_ids, k_d2)
            ev[4].record(stream)
            rcount(h, d_boxes, nb, cnt)
            ev[5].record(stream)
            if name not in rids:
                torch.cumsum(cnt, 0, out=off[1:])
                rids[name] = torch.empty(max(int(off[-1].item()), 1), dtype=torch.int32, device=dev)
                ev[5].record(stream)
            rreport(h, d_boxes, nb, off, rids[name])
            ev[6].record(stream)
            ev[6].synchronize()
            if it >= args.warmup:
                for j, p in enumerate(ms):
                    ms[p].append(ev[j].elapsed_time(ev[j + 1]))
        tr.sync()
        outs[name] = (k_ids.clone(), k_d2.clone(), cnt.clone())
        med = {p: round(float(np.median(v)), 3) for p, v in ms.items()}
        res[name] = {"ms": med, "build_mpts_s": round(n / med["build"] / 1e3, 1),
                     "insert_mpts_s": round(m / med["insert"] / 1e3, 1),
                     "delete_mpts_s": round(m / med["delete"] / 1e3, 1),
                     "knn_mq_s": round(nq / med["knn"] / 1e3, 1),
                     "range_count_mbox_s": round(nb / med["range_count"] / 1e3, 2),
                     "range_report_mbox_s": round(nb / med["range_report"] / 1e3, 2)}
        if name == "paper_shape":
            pn, root, ns, ls = tr.shape()
            res[name]["shape"] = {"points": pn, "node_slots": ns, "leaf_slots": ls}
        log(f"{name}: {res[name]}")
    a, b = outs["paper_shape"], outs["spac_h"]
    identical = all(bool(torch.equal(x, y)) for x, y in zip(a, b))
    ps, sp = res["paper_shape"], res["spac_h"]
    out = {"metric": "paper-shape SPaC-H build Mpoints/s (3D); join-based updates, kNN and range beside the "
                     "directory SPaC-H", "value": ps["build_mpts_s"],
           "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(sum(ps["ms"].values()), 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32/u64", "data": "synthetic",
           "config": {"workload": f"bst: {dim}D {args.dist} paper shape (leaf wrap 40) vs directory SPaC-H",
                      "n": n, "insert": m, "delete": m, "queries": nq, "k": k, "boxes": nb,
                      "leaf_size": args.leaf},
           "paper_shape": ps, "spac_h": sp,
           "spac_h_over_paper_shape": {p: round(ps["ms"][p] / sp["ms"][p], 3) for p in ps["ms"]},
           "knn_and_counts_identical": identical}
    print(json.dumps(out), flush=True)


def bench_multi(args):
    """Batched small indexes: one segmented build + one persistent kNN launch
    vs per-index builds and launches (and those launches replayed as a graph)."""
    import numpy as np
    import torch

    import paper_2601_05347_amd as psi
    import synth
    num = args.indexes
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)  # a created stream: the null stream cannot be captured
    with torch.cuda.stream(stream):
        _bench_multi(args, num, dev, stream, np, torch, psi, synth)


def _bench_multi(args, num, dev, stream, np, torch, psi, synth):
    r = synth.unit(synth.draws(synth.stream_key(args.seed, 77), 0, 2 * num))
    sizes = np.floor(10 ** (3 + 3 * r[:num])).astype(np.int64)
    qsizes = np.floor(10 ** (4 * r[num:])).astype(np.int64).clip(1, 10_000)
    t = time.perf_counter()
    pts = np.concatenate([synth.uniform(int(n), 2, 30, 1000 + i) for i, n in enumerate(sizes)])
    qs = np.concatenate([synth.uniform(int(n), 2, 30, 1000 + i, synth.P_QUERY) for i, n in enumerate(qsizes)])
    log(f"multi: {num} indexes, {len(pts)} points, {len(qs)} queries generated in {time.perf_counter() - t:.1f} s")
    off = np.concatenate(([0], np.cumsum(sizes))).astype(np.uint64)
    qoff = np.concatenate(([0], np.cumsum(qsizes))).astype(np.uint64)
    d_pts = torch.from_numpy(pts.view(np.int32)).to(dev)
    d_q = torch.from_numpy(qs.view(np.int32)).to(dev)
    d_off = torch.from_numpy(off.view(np.int64)).to(dev)
    d_qoff = torch.from_numpy(qoff.view(np.int64)).to(dev)
    k = 8
    ids = torch.empty((len(qs), k), dtype=torch.int32, device=dev)
    d2 = torch.empty((len(qs), k), dtype=torch.int64, device=dev)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best * 1e3

    holder = {}

    def multi_build():
        if "m" in holder:
            psi.psi_multi_destroy(holder.pop("m"))
        holder["m"] = psi.psi_multi_build(2, psi.MORTON, num, d_off, d_pts, args.leaf, args.fanout)

    t_mb = timed(multi_build)
    t_mk = timed(lambda: psi.psi_multi_knn(holder["m"], d_qoff, d_q, k, ids, d2))
    m_ids, m_d2 = ids.clone(), d2.clone()
    # per-index path: num separate indexes, num builds, num kNN calls
    singles = [psi.Index(2, psi.MORTON, args.leaf, args.fanout, device=dev) for _ in range(num)]
    pv = [d_pts[int(off[i]):int(off[i + 1])] for i in range(num)]
    qv = [d_q[int(qoff[i]):int(qoff[i + 1])] for i in range(num)]
    iv = [ids[int(qoff[i]):int(qoff[i + 1])] for i in range(num)]
    dv = [d2[int(qoff[i]):int(qoff[i + 1])] for i in range(num)]

    def single_build():
        for i in range(num):
            psi.psi_build(singles[i]._h, pv[i], int(sizes[i]))

    def single_knn():
        for i in range(num):
            psi.psi_knn(singles[i]._h, qv[i], int(qsizes[i]), k, iv[i], dv[i])

    t_sb = timed(single_build)
    t_sk = timed(single_knn)
    same = bool(torch.equal(ids, m_ids) and torch.equal(d2, m_d2))
    # the per-index launches captured once and replayed as one hipGraph
    psi.psi_graph_begin(stream)
    single_knn()
    g = psi.psi_graph_end(stream)
    t_gk = timed(lambda: psi.psi_graph_launch(g, stream))
    same_g = bool(torch.equal(ids, m_ids) and torch.equal(d2, m_d2))
    psi.psi_graph_destroy(g)
    out = {"metric": "batched small indexes: build points/s and kNN queries/s, one persistent launch",
           "value": round(len(qs) / (t_mk / 1e3), 1), "unit": "queries/s", "n_gpus": 1, "steps": 3, "warmup": 1,
           "ms_per_step": round(t_mb + t_mk, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32/u64", "data": "synthetic",
           "config": {"workload": "multi: 2D SPaC-Z, sizes log-uniform 1e3..1e6, queries 1..1e4, k=8",
                      "indexes": num, "points": int(len(pts)), "queries": int(len(qs))},
           "multi": {"build_ms": round(t_mb, 3), "knn_ms": round(t_mk, 3),
                     "build_mpts_s": round(len(pts) / t_mb / 1e3, 1)},
           "per_index": {"build_ms": round(t_sb, 3), "knn_ms": round(t_sk, 3), "knn_graph_ms": round(t_gk, 3)},
           "results_identical": same and same_g}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "multi":
        return bench_multi(args)
    if args.workload == "incr":
        return bench_incr(args)
    if args.workload in ("orth", "orth2d"):
        return bench_orth(args)
    if args.workload == "bst":
        return bench_bst(args)
    import numpy as np
    import torch

    import paper_2601_05347_amd as psi
    import synth

    cfg = dict(WORKLOADS[args.workload])
    if args.n:
        cfg["n"] = args.n
    if args.k:
        cfg["k"] = args.k
    dim, bits, n, m, nq, k, nb = (cfg[x] for x in ("dim", "bits", "n", "m", "nq", "k", "nb"))
    curve = psi.HILBERT if args.curve == "hilbert" else psi.MORTON
    ops = set(args.ops.split(","))
    dev = torch.device("cuda:0")

    t_gen = time.perf_counter()
    data, ins, q = synth.workload(args.dist, dim, bits, args.seed, n=n, n_insert=m, n_query=nq)
    dels = synth.delete_ids(np.arange(n + m, dtype=np.uint32), m, args.seed)
    centres = q[:nb] if len(q) >= nb else synth.uniform(nb, dim, bits, args.seed, synth.P_AUX)
    boxes = synth.boxes(centres, bits, args.seed)
    log(f"inputs generated in {time.perf_counter() - t_gen:.1f} s")
    d_data = torch.from_numpy(data.view(np.int32)).to(dev)
    d_ins = torch.from_numpy(ins.view(np.int32)).to(dev)
    d_dels = torch.from_numpy(dels.view(np.int32)).to(dev)
    d_q = torch.from_numpy(q.view(np.int32)).to(dev)
    d_boxes = torch.from_numpy(boxes.view(np.int32)).to(dev)
    del ins  # the points, queries and boxes stay on the host for the CPU baseline
    stream = torch.cuda.current_stream(dev)
    ix = psi.Index(dim, curve, args.leaf, args.fanout, device=dev, stream=stream,
                   flags=psi.FLAG_SORTED_LEAVES if args.sorted_leaves else 0)
    h = ix._h
    new_ids = torch.empty(m, dtype=torch.int32, device=dev)
    nd = torch.zeros(1, dtype=torch.int64, device=dev)
    k_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    k_d2 = torch.empty((nq, k), dtype=torch.int64, device=dev)
    r_cnt = torch.empty(nb, dtype=torch.int64, device=dev)
    r_off = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
    r_ids = None

    phases = ["build", "insert", "delete", "knn", "range_count", "range_report"]
    if "build" not in ops:  # the other phases still need an index: build it once, untimed
        psi.psi_build(h, d_data, n)
        ix.sync()

    def step(ev):
        nonlocal r_ids
        ev["build"][0].record(stream)
        if "build" in ops:
            psi.psi_build(h, d_data, n)
        ev["build"][1].record(stream)
        ev["insert"][0].record(stream)
        if "insert" in ops:
            psi.psi_batch_insert(h, d_ins, m, new_ids)
        ev["insert"][1].record(stream)
        ev["delete"][0].record(stream)
        if "delete" in ops:
            psi.psi_batch_delete(h, d_dels, m, nd)
        ev["delete"][1].record(stream)
        ev["knn"][0].record(stream)
        if "knn" in ops:
            psi.psi_knn(h, d_q, nq, k, k_ids, k_d2)
        ev["knn"][1].record(stream)
        ev["range_count"][0].record(stream)
        if "range" in ops:
            psi.psi_range_count(h, d_boxes, nb, r_cnt)
        ev["range_count"][1].record(stream)
        ev["range_report"][0].record(stream)
        if "range" in ops:
            torch.cumsum(r_cnt, 0, out=r_off[1:])
            if r_ids is None:  # sized once, from the first (untimed) step
                r_ids = torch.empty(max(1, int(r_off[-1].item())), dtype=torch.int32, device=dev)
            psi.psi_range_report(h, d_boxes, nb, r_off, r_ids)
        ev["range_report"][1].record(stream)

    def events():
        return {p: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for p in phases}

    # A plain device copy of known size (1 GiB read + 1 GiB written), outside
    # the timed region: rocprofv3 counter runs scale FETCH_SIZE / WRITE_SIZE
    # of the other kernels by what the counters read for this copy.
    calib_src = torch.ones(CALIB_BYTES // 4, dtype=torch.int32, device=dev)
    calib_dst = torch.empty_like(calib_src)
    calib_dst.copy_(calib_src)
    del calib_src, calib_dst

    for _ in range(max(args.warmup, 1 if "range" in ops else 0)):
        step(events())
    ix.sync()
    log("warmup done")
    # Two untimed steps with every kernel family bracketed by HIP events give
    # the per-family times and pick the dominant streaming kernel of the build
    # and update path; in the timed steps only that family is bracketed (its
    # launch time for the roofline), so the other events cost the timed
    # region nothing.
    fams = ["radix_first", "radix_pass", "bucket_starts", "local_sort", "local_sort_wide", "local_sort_huge", "radix_big",
            "encode_hist",
            "leaf_fill", "nodes", "hist",
            "radix_update", "radix_order", "order", "knn", "range_count", "range_report", "update"]
    PROF_STEPS = 2
    ix.prof_enable(True)
    ix.prof_reset()
    for _ in range(PROF_STEPS):
        step(events())
    prof = {f: ix.prof_get(f) for f in fams}
    mem_fams = [f for f in ("radix_first", "radix_pass", "local_sort", "radix_big", "encode_hist", "leaf_fill", "nodes")
                if prof[f][1] > 0 and prof[f][2] > 0]
    dom = max(mem_fams, key=lambda f: prof[f][0]) if mem_fams else None
    kernel_ms = {f: round(prof[f][0] / PROF_STEPS, 3) for f in fams if prof[f][1]}
    ix.prof_only(dom)
    ix.prof_enable(dom is not None)
    ix.prof_reset()
    evs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e = events()
        step(e)
        evs.append(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ix.sync()
    log(f"{args.steps} timed steps done in {wall:.2f} s")
    ms = {p: float(np.mean([e[p][0].elapsed_time(e[p][1]) for e in evs])) for p in phases}
    upd_ms = ms["build"] + ms["insert"] + ms["delete"]
    upd_pts = (n if "build" in ops else 0) + (m if "insert" in ops else 0) + (m if "delete" in ops else 0)
    value = upd_pts / (upd_ms / 1e3) / 1e6 if upd_ms > 0 else 0.0

    # the dominant kernel's roofline, from its launches in the timed steps
    roof = None
    tms, launches, byt = ix.prof_get(dom) if dom else (0.0, 0, 0)
    ix.prof_only(None)
    ix.prof_enable(False)
    if launches:
        avg_s = tms / launches / 1e3
        achieved = byt / launches / avg_s / 1e9
        traffic = None
        if args.workload == "3d-1e8" and args.dist == "uniform" and n == 100_000_000 and curve == 1:
            traffic = profiled_traffic("build_kernels_3d_1e8_uniform.md", dom)
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": byt // launches, "avg_launch_ms": round(tms / launches, 4)}

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} {args.dist} SPaC-{'H' if curve else 'Z'}", "n": n, "dim": dim,
                   "coord_bits": bits, "insert": m, "delete": m, "queries": nq, "k": k, "boxes": nb,
                   "leaf_size": args.leaf, "fanout": args.fanout, "ops": sorted(ops),
                   **({"sorted_leaves": True} if args.sorted_leaves else {})},
        "phases": {
            **{f"{p}_ms": round(v, 3) for p, v in ms.items()},
            "build_mpts_s": round(n / ms["build"] / 1e3, 1) if ms["build"] > 0 else None,
            "insert_mpts_s": round(m / ms["insert"] / 1e3, 1) if ms["insert"] > 0 and "insert" in ops else None,
            "delete_mpts_s": round(m / ms["delete"] / 1e3, 1) if ms["delete"] > 0 and "delete" in ops else None,
            "knn_queries_s": round(nq / ms["knn"] * 1e3, 0) if ms["knn"] > 0 and "knn" in ops else None,
            "range_count_boxes_s": round(nb / ms["range_count"] * 1e3, 0) if "range" in ops else None,
            "range_report_boxes_s": round(nb / ms["range_report"] * 1e3, 0) if "range" in ops else None,
            "range_report_ids": int(r_off[-1].item()) if "range" in ops else None,
        },
        "kernel_ms_per_step": kernel_ms,
        "roofline": roof,
    }
    if "knn" in ops:  # one more, untimed kNN pass with the walk counted
        psi.psi_query_stats(h, True)
        psi.psi_knn(h, d_q, nq, k, k_ids, k_d2)
        wc = psi.psi_query_stats(h, False).astype(np.float64)
        if wc[0] > 0:
            out["knn_walk"] = {"box_tests_per_query": round(wc[1] / wc[0], 2),
                               "leaves_per_query": round(wc[2] / wc[0], 2),
                               "points_per_query": round(wc[3] / wc[0], 2),
                               "touched_bytes_per_query": round((16 * wc[1] + 8 * wc[2] + 4 * (dim + 1) * wc[3]) / wc[0], 1)}
    if "knn" in ops and args.workload == "3d-1e8":
        # the configuration's other k: the same queries on the same (updated)
        # index, one untimed pass, then the mean of two passes (HIP events)
        out["knn_other_k"] = {}
        for kk in (1, 100):
            if kk == k:
                continue
            o_ids = torch.empty(nq * kk, dtype=torch.int32, device=dev)
            o_d2 = torch.empty(nq * kk, dtype=torch.int64, device=dev)
            psi.psi_knn(h, d_q, nq, kk, o_ids, o_d2)
            tms = []
            for _ in range(2):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                psi.psi_knn(h, d_q, nq, kk, o_ids, o_d2)
                b.record(stream)
                b.synchronize()
                tms.append(a.elapsed_time(b))
            kms = float(np.mean(tms))
            out["knn_other_k"][str(kk)] = {"ms": round(kms, 3), "queries_s": round(nq / kms * 1e3, 0)}
            del o_ids, o_d2
        log(f"kNN at other k: {out['knn_other_k']}")
    ix.close()
    del d_data, d_ins, d_dels, d_q, d_boxes, k_ids, k_d2, r_ids
    torch.cuda.empty_cache()
    if not args.no_serve and args.workload == "3d-1e8":
        scfg = WORKLOADS["serve"]
        log("serving block ...")
        lam_plain, runs = serve_runs(scfg["n"], args.serve_requests, [1.2], args.seed, args.leaf, args.fanout,
                                     paths=("plain", "library"))
        r = runs["rho=1.2"]
        out["serve"] = {"workload": f"resident 3D SPaC-H, {scfg['n']} uniform points, {args.serve_requests} "
                                    "Poisson requests 40/20/30/10 insert/delete/knn/range at 1.2x plain capacity",
                        "plain_capacity_req_s": round(lam_plain, 2),
                        **{name: {"p50_ms": round(r[name]["all"]["p50_ms"], 2), "p99_ms": round(r[name]["all"]["p99_ms"], 2),
                                  "throughput_req_s": round(r[name]["throughput_req_s"], 2)} for name in r}}
    if not args.no_cpu:
        log("timing the oracle on a CPU sample ...")
        out["cpu_baseline"] = cpu_baseline(cfg, args, full=(data, q, boxes, k) if "knn" in ops else None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
