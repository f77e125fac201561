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
    serve.BatchServer(ix, budget_bytes=budget).run(batch, realtime=False)
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
