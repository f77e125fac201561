"""Serving loop for a resident index: continuous batching of mixed requests.

Requests (insert, delete, kNN, range report) arrive over time. The plain
path (`PlainServer`) runs them one at a time in arrival order, each on its
own launches, waiting for each to finish. `BatchServer` serves them by
continuous batching:

* admission: arrived requests enter in arrival order while their estimated
  device footprint fits the HBM budget; their payloads are copied to the
  device on a separate stream as soon as they are admitted, overlapping the
  work already running;
* epochs: the head of the admitted queue is cut into maximal runs of one
  class. A run of updates is applied in order, consecutive inserts merged
  into one batch (ids are assigned in arrival order, so merging changes no
  id). A run of queries is fused: all kNN requests with the same k become one
  launch, all range requests one count and one report launch;
* consistency: every request sees exactly the updates that arrived before
  it, as if the requests ran one by one in arrival order.

`DeviceServer` does the same through the library's server (psi_server_*):
admission, epochs and the fusion of updates and kNN batches happen in the
C++ runtime, updates and queries run on two streams, and an update's batch
sort and routing overlap the queries of the epoch before it. This module
then only stages payloads and submits and polls requests.

Latency of a request = completion (a HIP event after its epoch) minus its
scheduled arrival. The index is the library's (all work runs in its HIP
kernels); this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np

from . import (REQ_DELETE, REQ_INSERT, REQ_KNN, REQ_RANGE_REPORT, Index, PsiError, psi_batch_delete, psi_batch_insert,
               psi_knn, psi_range_count, psi_range_report, psi_server_create, psi_server_destroy, psi_server_poll,
               psi_server_submit, psi_server_wait, to_u32, to_u64)

UPDATE, QUERY = 0, 1
KIND_CLASS = {"insert": UPDATE, "delete": UPDATE, "knn": QUERY, "range": QUERY}


def footprint(req: dict, dim: int) -> int:
    """Estimated device bytes a request holds while in flight."""
    k = req["kind"]
    if k == "insert":
        return len(req["points"]) * (4 * dim + 64)
    if k == "delete":
        return len(req["ids"]) * 64
    if k == "knn":
        return len(req["queries"]) * (4 * dim + 12 * req.get("k", 10) + 32)
    return len(req["boxes"]) * (8 * dim + 16 + 4096)  # report output estimated at 1k ids per box


def percentiles(lat_ms):
    if not lat_ms:
        return {"n": 0}
    a = np.sort(np.asarray(lat_ms))
    return {"n": int(a.size), "p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean())}


def summarize(reqs) -> dict:
    out = {}
    for kind in ("insert", "delete", "knn", "range"):
        out[kind] = percentiles([r["latency_ms"] for r in reqs if r["kind"] == kind and "latency_ms" in r])
    done = [r for r in reqs if "done_s" in r]
    if done:
        span = max(r["done_s"] for r in done) - min(r["arrival"] for r in done)
        out["throughput_req_s"] = len(done) / span if span > 0 else float("inf")
        out["all"] = percentiles([r["latency_ms"] for r in done])
    out["rejected"] = sum(1 for r in reqs if r.get("rejected"))
    return out


class _Clock:
    """Host clock aligned with a HIP event recorded at the same instant."""

    def __init__(self, stream):
        import torch
        self.torch = torch
        self.stream = stream
        stream.synchronize()
        self.base = torch.cuda.Event(enable_timing=True)
        self.base.record(stream)
        self.base.synchronize()
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def event(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        return e

    def seconds(self, ev) -> float:
        ev.synchronize()
        return self.base.elapsed_time(ev) / 1e3


def _wait_until(clock: _Clock, t: float):
    while True:
        d = t - clock.now()
        if d <= 0:
            return
        time.sleep(min(d, 2e-4))


class PlainServer:
    """One request at a time, in arrival order, each waited for."""

    def __init__(self, index: Index):
        self.ix = index

    def run(self, reqs, realtime: bool = True):
        import torch
        ix, dev, stream = self.ix, self.ix.device, self.ix.stream
        clock = _Clock(stream)
        for r in reqs:
            if realtime:
                _wait_until(clock, r["arrival"])
            with torch.cuda.stream(stream):
                r["result"] = _execute_one(ix, r, dev)
            ev = clock.event()
            r["done_s"] = clock.seconds(ev)
            r["latency_ms"] = (r["done_s"] - r["arrival"]) * 1e3
        return reqs


def _execute_one(ix: Index, r: dict, dev):
    k = r["kind"]
    if k == "insert":
        return to_u32(ix.batch_insert(r["points"]))
    if k == "delete":
        return int(to_u64(ix.batch_delete(r["ids"]))[0])
    if k == "knn":
        ids, d2 = ix.knn(r["queries"], r.get("k", 10))
        return to_u32(ids), to_u64(d2)
    off, ids = ix.range_report(r["boxes"])
    return to_u64(off), to_u32(ids)


def _fetch(r):
    """Host copy of a finished request's result (after its epoch's event)."""
    res = r.pop("result_dev")
    k = r["kind"]
    if k == "insert":
        return to_u32(res)
    if k == "delete":
        return int(to_u64(res)[0])
    if k == "knn":
        return to_u32(res[0]), to_u64(res[1])
    off = to_u64(res[0])
    base = int(off[0])
    return (off - np.uint64(base)).astype(np.uint64), to_u32(res[1][base:int(off[-1])])


class _PinnedRing:
    """Pinned host staging area allocated once: payloads are copied into it
    and uploaded from it asynchronously; space is reused once the upload that
    read it has completed (events checked oldest first)."""

    def __init__(self, nbytes: int):
        import torch
        self.buf = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        self.np = self.buf.numpy()
        self.size = nbytes
        self.head = 0
        self.live = deque()  # (start, end, event) of uploads in flight

    def _reclaim(self, block: bool):
        while self.live and (block or self.live[0][2].query()):
            self.live[0][2].synchronize()
            self.live.popleft()
            block = False

    def take(self, n: int):
        """Offset of n free bytes (n <= size), 256-aligned."""
        n = (n + 255) & ~255
        while True:
            self._reclaim(False)
            start = self.head if self.head + n <= self.size else 0
            end = start + n
            if all(e <= start or s >= end for s, e, _ in self.live):
                self.head = end
                return start
            self._reclaim(True)

    def done(self, start: int, n: int, event):
        self.live.append((start, start + ((n + 255) & ~255), event))


class BatchServer:
    """Continuous batching with HBM-budget admission (see module docstring)."""

    def __init__(self, index: Index, budget_bytes: int = 32 << 30, staging_bytes: int = 64 << 20):
        import torch
        self.ix = index
        self.budget = budget_bytes
        self.copy_stream = torch.cuda.Stream(device=index.device)
        self.ring = _PinnedRing(staging_bytes)

    # payload upload on the copy stream; compute waits on the event
    def _stage(self, r):
        import torch
        dev = self.ix.device
        arr = r.get("points", r.get("ids", r.get("queries", r.get("boxes"))))
        a = np.ascontiguousarray(arr)
        a = a.view(np.int32) if a.dtype == np.uint32 else a
        nb = a.nbytes
        if nb == 0 or nb > self.ring.size:  # too large to stage: plain pinned copy
            host = torch.from_numpy(a).pin_memory()
            r["_host"] = host
        else:
            off = self.ring.take(nb)
            self.ring.np[off:off + nb] = a.reshape(-1).view(np.uint8)
            host = self.ring.buf[off:off + nb].view(torch.int32 if a.dtype == np.int32 else torch.int64)
        with torch.cuda.stream(self.copy_stream):
            r["dev"] = host.to(dev, non_blocking=True).reshape(a.shape)
            r["ready"] = torch.cuda.Event()
            r["ready"].record(self.copy_stream)
        if 0 < nb <= self.ring.size:
            self.ring.done(off, nb, r["ready"])

    def run(self, reqs, realtime: bool = True):
        import torch
        ix = self.ix
        dev, stream, D = ix.device, ix.stream, ix.dim
        h = ix._h
        clock = _Clock(stream)
        pending = deque(reqs)
        queue = deque()
        in_flight = 0
        self.max_in_flight = 0
        epochs = []  # (event, requests) awaiting completion times

        def admit():
            nonlocal in_flight
            while pending and (not realtime or pending[0]["arrival"] <= clock.now()):
                r = pending[0]
                fp = footprint(r, D)
                if fp > self.budget:  # can never fit: rejected at admission
                    pending.popleft()
                    r["rejected"] = True
                    continue
                if in_flight + fp > self.budget:
                    if queue:  # serve what is admitted first
                        break
                    if epochs:  # wait for the oldest epoch to free its share, then retry
                        finish([epochs.pop(0)])
                        continue
                pending.popleft()
                r["fp"] = fp
                in_flight += fp
                self.max_in_flight = max(self.max_in_flight, in_flight)
                self._stage(r)
                queue.append(r)

        def finish(done_epochs):
            nonlocal in_flight
            for ev, group in done_epochs:
                t = clock.seconds(ev)
                for r in group:
                    r["done_s"] = t
                    r["latency_ms"] = (t - r["arrival"]) * 1e3
                    in_flight -= r.get("fp", 0)
                    r["result"] = _fetch(r)
                    r.pop("dev", None)
                    r.pop("_host", None)

        while pending or queue:
            admit()
            if not queue:
                if pending and realtime:
                    _wait_until(clock, pending[0]["arrival"])
                continue
            cls = KIND_CLASS[queue[0]["kind"]]
            group = []
            while queue and KIND_CLASS[queue[0]["kind"]] == cls:
                group.append(queue.popleft())
            with torch.cuda.stream(stream):
                for r in group:
                    stream.wait_event(r["ready"])
                if cls == UPDATE:
                    self._updates(group, h, dev)
                else:
                    self._queries(group, h, dev)
                ev = clock.event()
            epochs.append((ev, group))
            # retire finished epochs so their budget frees up
            while len(epochs) > 1 and epochs[0][0].query():
                finish([epochs.pop(0)])
        finish(epochs)
        return reqs

    def _updates(self, group, h, dev):
        import torch
        i = 0
        while i < len(group):
            r = group[i]
            if r["kind"] == "insert":
                j = i
                while j < len(group) and group[j]["kind"] == "insert":
                    j += 1
                pts = torch.cat([g["dev"].reshape(-1, self.ix.dim) for g in group[i:j]]) if j - i > 1 else \
                    r["dev"].reshape(-1, self.ix.dim)
                m = pts.shape[0]
                new_ids = torch.empty(m, dtype=torch.int32, device=dev)
                psi_batch_insert(h, pts, m, new_ids)
                o = 0
                for g in group[i:j]:
                    n = len(g["points"])
                    g["result_dev"] = new_ids[o:o + n]
                    o += n
                i = j
            else:
                nd = torch.zeros(1, dtype=torch.int64, device=dev)
                psi_batch_delete(h, r["dev"], len(r["ids"]), nd)
                r["result_dev"] = nd
                i += 1

    def _queries(self, group, h, dev):
        import torch
        D = self.ix.dim
        by_k = {}
        for r in group:
            if r["kind"] == "knn":
                by_k.setdefault(r.get("k", 10), []).append(r)
        for k, rs in by_k.items():
            q = torch.cat([r["dev"].reshape(-1, D) for r in rs]) if len(rs) > 1 else rs[0]["dev"].reshape(-1, D)
            nq = q.shape[0]
            ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
            d2 = torch.empty((nq, k), dtype=torch.int64, device=dev)
            psi_knn(h, q, nq, k, ids, d2)
            o = 0
            for r in rs:
                n = len(r["queries"])
                r["result_dev"] = (ids[o:o + n], d2[o:o + n])
                o += n
        rr = [r for r in group if r["kind"] == "range"]
        if rr:
            b = torch.cat([r["dev"].reshape(-1, 2, D) for r in rr]) if len(rr) > 1 else rr[0]["dev"].reshape(-1, 2, D)
            nb = b.shape[0]
            cnt = torch.empty(nb, dtype=torch.int64, device=dev)
            psi_range_count(h, b, nb, cnt)
            off = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
            torch.cumsum(cnt, 0, out=off[1:])
            total = int(off[-1].item())
            out = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
            psi_range_report(h, b, nb, off, out)
            o = 0
            for r in rr:
                n = len(r["boxes"])
                r["result_dev"] = (off[o:o + n + 1], out)
                o += n


class DeviceServer:
    """Continuous batching by the library's server (psi_server_*): this class
    stages each request's payload on a copy stream, submits it with the
    upload's event, and polls for completion; admission, epochs, fusion and
    the overlap of updates with queries happen in the C++ runtime."""

    def __init__(self, index: Index, budget_bytes: int = 32 << 30, staging_bytes: int = 64 << 20,
                 report_slack: float = 4.0):
        import torch
        self.ix = index
        self.budget = budget_bytes
        self.copy_stream = torch.cuda.Stream(device=index.device)
        self.ring = _PinnedRing(staging_bytes)
        self.report_slack = report_slack
        self.n_live = None

    _stage = BatchServer._stage

    def _report_capacity(self, boxes, n_live: int, bits: int) -> int:
        """Output room for a range report: the expected hits of each box under
        a uniform density (n_live points in [0, 2^bits)^dim), times a slack,
        plus a margin; a box past the room is truncated and reported as such."""
        b = np.asarray(boxes, dtype=np.float64).reshape(len(boxes), 2, -1)
        vol = np.prod(np.maximum(b[:, 1] - b[:, 0] + 1, 0), axis=1) / float(1 << bits) ** b.shape[2]
        return int(self.report_slack * float(vol.sum()) * n_live) + 1024 * len(boxes) + 1024

    def run(self, reqs, realtime: bool = True, n_live: int = 0, bits: int = 21):
        import torch
        ix = self.ix
        dev, D = ix.device, ix.dim
        srv = psi_server_create(ix._h, self.budget)
        t0 = time.perf_counter()  # the server's clock starts at creation (its base event has completed)
        live = n_live
        outstanding = deque()
        try:
            i = 0
            while i < len(reqs) or outstanding:
                now = time.perf_counter() - t0
                while i < len(reqs) and (not realtime or reqs[i]["arrival"] <= now):
                    r = reqs[i]
                    i += 1
                    self._stage(r)
                    k = r["kind"]
                    if k == "insert":
                        n = len(r["points"])
                        r["out"] = (torch.empty(max(n, 1), dtype=torch.int32, device=dev),)
                        r["ticket"] = psi_server_submit(srv, REQ_INSERT, n, r["dev"], d_ids=r["out"][0],
                                                        ready_event=r["ready"])
                        live += n
                    elif k == "delete":
                        n = len(r["ids"])
                        # written by the delete itself (a fill here would run on another
                        # stream, unordered with the server's write)
                        r["out"] = (torch.empty(1, dtype=torch.int64, device=dev),)
                        r["ticket"] = psi_server_submit(srv, REQ_DELETE, n, r["dev"], d_out=r["out"][0],
                                                        ready_event=r["ready"])
                        live -= n
                    elif k == "knn":
                        n, kk = len(r["queries"]), r.get("k", 10)
                        r["out"] = (torch.empty((max(n, 1), kk), dtype=torch.int32, device=dev),
                                    torch.empty((max(n, 1), kk), dtype=torch.int64, device=dev))
                        r["ticket"] = psi_server_submit(srv, REQ_KNN, n, r["dev"], d_ids=r["out"][0],
                                                        d_out=r["out"][1], k=kk, ready_event=r["ready"])
                    else:
                        n = len(r["boxes"])
                        cap = self._report_capacity(r["boxes"], max(live, 1), bits)
                        r["out"] = (torch.empty(n + 1, dtype=torch.int64, device=dev),
                                    torch.empty(cap, dtype=torch.int32, device=dev))
                        r["cap"] = cap
                        r["ticket"] = psi_server_submit(srv, REQ_RANGE_REPORT, n, r["dev"], d_ids=r["out"][1],
                                                        d_out=r["out"][0], ids_cap=cap, ready_event=r["ready"])
                    outstanding.append(r)
                # completions, oldest first, up to the first ticket still running
                # (each poll also dispatches what is queued; the completion time is
                # the server's event time, so a ticket collected late is timed right)
                while outstanding:
                    r = outstanding[0]
                    try:
                        done, ms = psi_server_poll(srv, r["ticket"])
                    except PsiError as e:
                        if e.code != 4:  # PSI_E_CAPACITY: a request larger than the whole budget
                            raise
                        r["rejected"] = True
                        r.pop("out", None)
                        outstanding.popleft()
                        continue
                    if not done:
                        break
                    self._finish(r, ms)
                    outstanding.popleft()
                if outstanding or i < len(reqs):
                    nxt = reqs[i]["arrival"] if i < len(reqs) and realtime else None
                    if not outstanding and nxt is not None:
                        time.sleep(max(0.0, min(nxt - (time.perf_counter() - t0), 2e-4)))
                    elif outstanding:
                        time.sleep(5e-5)
        finally:
            for r in outstanding:
                try:
                    self._finish(r, psi_server_wait(srv, r["ticket"]))
                except PsiError as e:
                    if e.code != 4:
                        raise
                    r["rejected"] = True
            psi_server_destroy(srv)
        return reqs

    def _finish(self, r, ms):
        r["done_s"] = ms / 1e3
        r["latency_ms"] = (r["done_s"] - r["arrival"]) * 1e3
        out = r.pop("out")
        k = r["kind"]
        if k == "insert":
            r["result"] = to_u32(out[0][:len(r["points"])])
        elif k == "delete":
            r["result"] = int(to_u64(out[0])[0])
        elif k == "knn":
            n = len(r["queries"])
            r["result"] = (to_u32(out[0][:n]), to_u64(out[1][:n]))
        else:
            off = to_u64(out[0])
            total = int(off[-1])
            r["truncated"] = total > r["cap"]
            r["result"] = (off, to_u32(out[1][:min(total, r["cap"])]))
        r.pop("dev", None)
        r.pop("_host", None)
