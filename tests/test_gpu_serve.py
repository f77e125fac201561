"""Serving loop: every request's result under continuous batching equals the
result of running the requests one at a time in arrival order (the oracle,
and the plain per-request path). Exact: everything is integer."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_replay(dim, curve, base, reqs):
    ref = oracle.RefIndex(dim, curve, 32, 8)
    ref.build(base)
    out = []
    for r in reqs:
        k = r["kind"]
        if k == "insert":
            out.append(ref.batch_insert(r["points"]))
        elif k == "delete":
            out.append(ref.batch_delete(r["ids"]))
        elif k == "knn":
            out.append(ref.knn(r["queries"], r.get("k", 10)))
        else:
            out.append(ref.range_report(r["boxes"]))
    return out


def same(kind, got, exp):
    if kind == "insert":
        np.testing.assert_array_equal(got, exp)
    elif kind == "delete":
        assert got == exp, (got, exp)
    elif kind == "knn":
        np.testing.assert_array_equal(got[0], exp[0])
        np.testing.assert_array_equal(got[1], exp[1])
    else:
        goff, gids = got
        eoff, eids = exp
        np.testing.assert_array_equal(goff, eoff)
        for b in range(len(goff) - 1):
            np.testing.assert_array_equal(np.sort(gids[goff[b]:goff[b + 1]]), eids[eoff[b]:eoff[b + 1]])


@pytest.mark.parametrize("budget", [32 << 30, 2 << 20])
def test_batched_serving_matches_sequential(budget):
    import torch
    assert torch.cuda.is_available()
    import paper_2601_05347_amd as psi
    from paper_2601_05347_amd import serve
    say(f"serve budget={budget}")
    dim, curve = 3, 1
    base = synth.uniform(100_000, dim, 21, seed=5)
    reqs = synth.request_stream(300, len(base), dim, 21, seed=6, rate_per_s=1e6, upd_size=(10, 5000),
                                knn_size=(1, 2000), range_size=(1, 200))
    expected = oracle_replay(dim, curve, base, reqs)
    ix = psi.Index(dim, curve, 32, 8)
    ix.build(base)
    batch = [dict(r) for r in reqs]
    bs = serve.BatchServer(ix, budget_bytes=budget)
    bs.run(batch, realtime=False)
    # admission never holds more than the budget (a request fits it alone)
    assert bs.max_in_flight <= budget
    for r, e in zip(batch, expected):
        assert not r.get("rejected")
        same(r["kind"], r["result"], e)
    ix.sync()
    stats = serve.summarize(batch)
    assert stats["all"]["n"] == 300
    # the plain per-request path gives the same answers
    ix2 = psi.Index(dim, curve, 32, 8)
    ix2.build(base)
    plain = [dict(r) for r in reqs]
    serve.PlainServer(ix2).run(plain, realtime=False)
    for r, e in zip(plain, expected):
        same(r["kind"], r["result"], e)
    ix2.sync()


def test_realtime_arrivals_and_rejection():
    import torch
    assert torch.cuda.is_available()
    import paper_2601_05347_amd as psi
    from paper_2601_05347_amd import serve
    say("serve realtime")
    base = synth.uniform(50_000, 2, 30, seed=7)
    reqs = synth.request_stream(120, len(base), 2, 30, seed=8, rate_per_s=3000.0, upd_size=(10, 3000),
                                knn_size=(1, 500), range_size=(1, 50))
    big = {"kind": "knn", "arrival": reqs[-1]["arrival"] + 1e-3,
           "queries": synth.uniform(50_000, 2, 30, seed=9, purpose=synth.P_QUERY), "k": 10}
    reqs.append(big)
    expected = oracle_replay(2, 0, base, reqs[:-1])
    ix = psi.Index(2, 0, 32, 8)
    ix.build(base)
    # budget too small for the last request alone: it is rejected, the rest served
    out = serve.BatchServer(ix, budget_bytes=2 << 20).run([dict(r) for r in reqs], realtime=True)
    assert out[-1].get("rejected")
    for r, e in zip(out[:-1], expected):
        same(r["kind"], r["result"], e)
        assert r["latency_ms"] >= 0
    ix.sync()


@pytest.mark.parametrize("budget", [32 << 30, 2 << 20])
def test_library_server_matches_sequential(budget):
    """The C++ server (psi_server_*): epochs on two streams, updates
    overlapping the queries before them, same answers as one at a time."""
    import torch
    assert torch.cuda.is_available()
    import paper_2601_05347_amd as psi
    from paper_2601_05347_amd import serve
    say(f"library server budget={budget}")
    dim, curve = 3, 1
    base = synth.uniform(100_000, dim, 21, seed=15)
    reqs = synth.request_stream(300, len(base), dim, 21, seed=16, rate_per_s=1e6, upd_size=(10, 5000),
                                knn_size=(1, 2000), range_size=(1, 200))
    expected = oracle_replay(dim, curve, base, reqs)
    ix = psi.Index(dim, curve, 32, 8)
    ix.build(base)
    out = serve.DeviceServer(ix, budget_bytes=budget).run([dict(r) for r in reqs], realtime=False,
                                                         n_live=len(base), bits=21)
    for r, e in zip(out, expected):
        assert not r.get("rejected") and not r.get("truncated")
        same(r["kind"], r["result"], e)
        assert r["latency_ms"] >= 0
    ix.sync()
    # the index is the library's again, and holds the replayed set
    ref = oracle.RefIndex(dim, curve, 32, 8)
    ref.build(base)
    for r in reqs:
        if r["kind"] == "insert":
            ref.batch_insert(r["points"])
        elif r["kind"] == "delete":
            ref.batch_delete(r["ids"])
    for a, b in zip(ix.export(), ref.dump()):
        np.testing.assert_array_equal(a, b)


def test_library_server_realtime_and_rejection():
    import torch
    assert torch.cuda.is_available()
    import paper_2601_05347_amd as psi
    from paper_2601_05347_amd import serve
    say("library server realtime")
    base = synth.uniform(50_000, 2, 30, seed=17)
    reqs = synth.request_stream(150, len(base), 2, 30, seed=18, rate_per_s=3000.0, upd_size=(10, 3000),
                                knn_size=(1, 500), range_size=(1, 50))
    big = {"kind": "knn", "arrival": reqs[-1]["arrival"] + 1e-3,
           "queries": synth.uniform(50_000, 2, 30, seed=19, purpose=synth.P_QUERY), "k": 10}
    reqs.append(big)
    expected = oracle_replay(2, 0, base, reqs[:-1])
    ix = psi.Index(2, 0, 32, 8)
    ix.build(base)
    out = serve.DeviceServer(ix, budget_bytes=2 << 20).run([dict(r) for r in reqs], realtime=True,
                                                          n_live=len(base), bits=30)
    assert out[-1].get("rejected")
    for r, e in zip(out[:-1], expected):
        same(r["kind"], r["result"], e)
        assert r["latency_ms"] >= 0
    ix.sync()


@pytest.mark.slow
def test_library_server_at_5e7_points_equals_the_plain_path():
    """A replay sample at the serving configuration's size: 5e7 resident 3D
    points, the full request mix; every answer of the library server equals
    the plain one-at-a-time path's (itself checked against the oracle)."""
    import torch
    assert torch.cuda.is_available()
    import paper_2601_05347_amd as psi
    from paper_2601_05347_amd import serve
    say("library server at 5e7")
    dim, curve, bits = 3, 1, 21
    base = synth.uniform(50_000_000, dim, bits, seed=21)
    reqs = synth.request_stream(160, len(base), dim, bits, seed=22, rate_per_s=1e6)
    ix = psi.Index(dim, curve, 32, 8)
    ix.build(base)
    out = serve.DeviceServer(ix).run([dict(r) for r in reqs], realtime=False, n_live=len(base), bits=bits)
    ix.close()
    torch.cuda.synchronize()
    ix2 = psi.Index(dim, curve, 32, 8)
    ix2.build(base)
    plain = serve.PlainServer(ix2).run([dict(r) for r in reqs], realtime=False)
    for r, p in zip(out, plain):
        assert not r.get("truncated")
        if r["kind"] == "range":
            same(r["kind"], r["result"], (p["result"][0], np.concatenate(
                [np.sort(p["result"][1][p["result"][0][b]:p["result"][0][b + 1]])
                 for b in range(len(p["result"][0]) - 1)] + [np.zeros(0, np.uint32)])))
        else:
            same(r["kind"], r["result"], p["result"])
    ix2.sync()
