"""Build, insert and delete are queued without waiting, and can be captured.

The sizes of the tree (leaf count, directory buffer, slots, next id, node
layout) live on the device, so an update call returns before its work has
run, a whole build-update-query sequence replays from a hipGraph, and a
captured insert keeps handing out fresh ids on every replay. A graph taken
before an eager update is refused (it would read a stale directory), and a
batch with an out-of-range coordinate is rejected whole on the device.
"""
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from invariants import check

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def psi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2601_05347_amd as psi
    psi.lib()
    return psi


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to("cuda")


def test_update_calls_return_while_the_stream_is_busy(psi):
    import torch
    say("enqueue-only updates")
    stream = torch.cuda.Stream()
    data, ins, q = synth.workload("uniform", 3, 21, seed=31, n=2_000_000, n_insert=200_000, n_query=400_000)
    dels = synth.delete_ids(np.arange(2_000_000, dtype=np.uint32), 150_000, seed=32)
    with torch.cuda.stream(stream):
        ix = psi.Index(3, psi.HILBERT, 32, 8, stream=stream)
        dq, di, dd = _dev(q), _dev(ins), _dev(dels)
        ids = torch.empty((len(q), 16), dtype=torch.int32, device="cuda")
        d2 = torch.empty((len(q), 16), dtype=torch.int64, device="cuda")
        new = torch.empty(len(ins), dtype=torch.int32, device="cuda")
        nd = torch.zeros(1, dtype=torch.int64, device="cuda")
        ix.build(data)
        # one eager round sizes every buffer
        psi.psi_batch_insert(ix._h, di, len(ins), new)
        psi.psi_batch_delete(ix._h, dd, len(dels), nd)
        psi.psi_knn(ix._h, dq, len(q), 16, ids, d2)
        ix.build(data)
        stream.synchronize()
        # a long kNN first, then the updates: if a call waited for its own
        # work it would also wait for the kNN queued before it
        busy = []
        for _ in range(3):
            psi.psi_knn(ix._h, dq, len(q), 16, ids, d2)
            t0 = time.perf_counter()
            psi.psi_batch_insert(ix._h, di, len(ins), new)
            psi.psi_batch_delete(ix._h, dd, len(dels), nd)
            t1 = time.perf_counter()
            busy.append(not stream.query())
            stream.synchronize()
            ix.build(data)
            stream.synchronize()
            say(f"  insert + delete calls took {1e3 * (t1 - t0):.2f} ms of host time; stream busy: {busy[-1]}")
        assert all(busy)
        # and the queued work was right
        psi.psi_batch_insert(ix._h, di, len(ins), new)
        psi.psi_batch_delete(ix._h, dd, len(dels), nd)
        ref = oracle.RefIndex(3, psi.HILBERT, 32, 8)
        ref.build(data)
        ref.batch_insert(ins)
        assert int(psi.to_u64(nd)[0]) == ref.batch_delete(dels)
        ix.sync()
        for a, b in zip(ix.export(), ref.dump()):
            np.testing.assert_array_equal(a, b)


def _sequence(psi, h, dpts, n, dins, m, ddel, md, dq, nq, db, nb, new, nd, ids, d2, cnt):
    psi.psi_build(h, dpts, n)
    psi.psi_batch_insert(h, dins, m, new)
    psi.psi_batch_delete(h, ddel, md, nd)
    psi.psi_knn(h, dq, nq, 10, ids, d2)
    psi.psi_range_count(h, db, nb, cnt)


@pytest.mark.parametrize("dim,curve,phi", [(2, 0, 32), (3, 1, 17)])
def test_graph_of_build_updates_and_queries(psi, dim, curve, phi):
    import torch
    say(f"graph build+insert+delete+knn+range dim={dim} curve={curve} phi={phi}")
    bits = 30 if dim == 2 else 21
    data, ins, q = synth.workload("varden", dim, bits, seed=41, n=60_000, n_insert=25_000, n_query=3000)
    dels = synth.delete_ids(np.arange(85_000, dtype=np.uint32), 40_000, seed=42)
    bx = synth.boxes(q[:700], bits, seed=43, side_lo=8, side_hi=18)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ix = psi.Index(dim, curve, phi, 4, stream=stream)
        h = ix._h
        dpts, dins, ddel, dq, db = _dev(data), _dev(ins), _dev(dels), _dev(q), _dev(bx)
        new = torch.empty(len(ins), dtype=torch.int32, device="cuda")
        nd = torch.zeros(1, dtype=torch.int64, device="cuda")
        ids = torch.empty((len(q), 10), dtype=torch.int32, device="cuda")
        d2 = torch.empty((len(q), 10), dtype=torch.int64, device="cuda")
        cnt = torch.empty(len(bx), dtype=torch.int64, device="cuda")
        args = (h, dpts, len(data), dins, len(ins), ddel, len(dels), dq, len(q), db, len(bx), new, nd, ids, d2, cnt)
        # the eager run: the reference, and it sizes every buffer
        _sequence(psi, *args)
        ix.sync()
        eager = [t.clone() for t in (new, nd, ids, d2, cnt)]
        e_dump = ix.export()
        psi.psi_graph_begin(stream)
        _sequence(psi, *args)
        g = psi.psi_graph_end(stream)
        for rep in range(3):
            for t in (new, ids, d2, cnt):
                t.fill_(-1)
            nd.fill_(-1)
            psi.psi_graph_launch(g, stream)
            stream.synchronize()
            for a, b in zip((new, nd, ids, d2, cnt), eager):
                assert torch.equal(a, b), rep
            # eager work between replays (a query only: an eager update would
            # stale the graph)
            psi.psi_knn(h, dq, 100, 4, ids[:100, :4].contiguous(), d2[:100, :4].contiguous())
            stream.synchronize()
            for a, b in zip(ix.export(), e_dump):
                np.testing.assert_array_equal(a, b)
            check(ix, phi, 4, curve)
        psi.psi_graph_destroy(g)
    ref = oracle.RefIndex(dim, curve, phi, 4)
    ref.build(data)
    np.testing.assert_array_equal(psi.to_u32(eager[0]), ref.batch_insert(ins))
    assert int(psi.to_u64(eager[1])[0]) == ref.batch_delete(dels)
    for a, b in zip(e_dump, ref.dump()):
        np.testing.assert_array_equal(a, b)
    r_ids, r_d2 = ref.knn(q, 10)
    np.testing.assert_array_equal(psi.to_u32(eager[2]), r_ids)
    np.testing.assert_array_equal(psi.to_u64(eager[3]), r_d2)
    np.testing.assert_array_equal(psi.to_u64(eager[4]), ref.range_count(bx))


def test_graph_insert_replays_hand_out_fresh_ids(psi):
    import torch
    say("graph insert replays")
    data, ins, _ = synth.workload("uniform", 2, 30, seed=51, n=40_000, n_insert=6000, n_query=0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ix = psi.Index(2, psi.HILBERT, 32, 8, stream=stream)
        dins = _dev(ins)
        new = torch.empty(len(ins), dtype=torch.int32, device="cuda")
        # size the buffers for several inserts, then start again
        ix.build(data)
        for _ in range(4):
            psi.psi_batch_insert(ix._h, dins, len(ins), new)
        ix.build(data)
        ix.sync()
        psi.psi_graph_begin(stream)
        psi.psi_batch_insert(ix._h, dins, len(ins), new)
        g = psi.psi_graph_end(stream)
        ref = oracle.RefIndex(2, psi.HILBERT, 32, 8)
        ref.build(data)
        for rep in range(3):
            psi.psi_graph_launch(g, stream)
            stream.synchronize()
            np.testing.assert_array_equal(psi.to_u32(new), ref.batch_insert(ins))
        psi.psi_graph_destroy(g)
        ix.sync()
        assert ix.size() == ref.size() and ix.next_id() == ref.next_id()
        for a, b in zip(ix.export(), ref.dump()):
            np.testing.assert_array_equal(a, b)
        check(ix, 32, 8, psi.HILBERT)


def test_graph_is_refused_after_an_eager_update(psi):
    import torch
    say("stale graph refused")
    data, ins, q = synth.workload("uniform", 3, 21, seed=61, n=30_000, n_insert=5000, n_query=800)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ix = psi.Index(3, psi.HILBERT, 32, 8, stream=stream)
        ix.build(data)
        dq = _dev(q)
        ids = torch.empty((len(q), 10), dtype=torch.int32, device="cuda")
        d2 = torch.empty((len(q), 10), dtype=torch.int64, device="cuda")
        psi.psi_knn(ix._h, dq, len(q), 10, ids, d2)
        ix.sync()
        psi.psi_graph_begin(stream)
        psi.psi_knn(ix._h, dq, len(q), 10, ids, d2)
        g = psi.psi_graph_end(stream)
        psi.psi_graph_launch(g, stream)  # still current
        stream.synchronize()
        ix.batch_insert(ins)
        ix.sync()
        with pytest.raises(psi.PsiError) as e:
            psi.psi_graph_launch(g, stream)
        assert e.value.code == 6
        psi.psi_graph_destroy(g)
        # the refused launch queued nothing; the index answers as the oracle
        ref = oracle.RefIndex(3, psi.HILBERT, 32, 8)
        ref.build(data)
        ref.batch_insert(ins)
        g_ids, g_d2 = ix.knn(q, 10)
        r_ids, r_d2 = ref.knn(q, 10)
        np.testing.assert_array_equal(psi.to_u32(g_ids), r_ids)
        np.testing.assert_array_equal(psi.to_u64(g_d2), r_d2)


def test_update_needing_more_room_is_refused_under_capture(psi):
    import torch
    say("capture refuses growth")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ix = psi.Index(2, 0, 32, 8, stream=stream)
        ix.build(synth.uniform(1000, 2, 30, seed=1))
        pts = _dev(synth.uniform(200_000, 2, 30, seed=2))
        ix.sync()
        psi.psi_graph_begin(stream)
        with pytest.raises(psi.PsiError) as e:
            psi.psi_batch_insert(ix._h, pts, 200_000)
        g = psi.psi_graph_end(stream)
        psi.psi_graph_destroy(g)
        assert e.value.code == 6
        ix.sync()
        assert ix.size() == 1000


@pytest.mark.parametrize("dim", [2, 3])
def test_out_of_range_insert_is_rejected_whole(psi, dim):
    say(f"rejected insert dim={dim}")
    bits = 30 if dim == 2 else 21
    data = synth.uniform(5000, dim, bits, seed=71)
    ix = psi.Index(dim, psi.HILBERT, 32, 8)
    ix.build(data)
    before = ix.export()
    bad = synth.uniform(3000, dim, bits, seed=72)
    bad[1234, dim - 1] = (1 << 31) if dim == 2 else (1 << 21)
    new = ix.batch_insert(bad)
    with pytest.raises(psi.PsiError) as e:
        ix.sync()
    assert e.value.code == 2
    assert (psi.to_u32(new) == 0xFFFFFFFF).all()
    assert ix.size() == 5000 and ix.next_id() == 5000
    for a, b in zip(ix.export(), before):
        np.testing.assert_array_equal(a, b)
    # the index goes on as before: the next batch gets ids 5000..
    good = synth.uniform(700, dim, bits, seed=73)
    np.testing.assert_array_equal(psi.to_u32(ix.batch_insert(good)), np.arange(5000, 5700, dtype=np.uint32))
    ix.sync()
    ref = oracle.RefIndex(dim, psi.HILBERT, 32, 8)
    ref.build(data)
    ref.batch_insert(good)
    for a, b in zip(ix.export(), ref.dump()):
        np.testing.assert_array_equal(a, b)


def test_odd_leaf_size_keeps_leaves_within_two_phi(psi):
    say("odd phi occupancy")
    phi = 17
    data, ins, _ = synth.workload("varden", 2, 30, seed=81, n=20_000, n_insert=40_000, n_query=0)
    ix = psi.Index(2, psi.MORTON, phi, 4)
    ref = oracle.RefIndex(2, psi.MORTON, phi, 4)
    ix.build(data)
    ref.build(data)
    for part in np.array_split(ins, 8):
        np.testing.assert_array_equal(psi.to_u32(ix.batch_insert(part)), ref.batch_insert(part))
        ix.sync()
        st = check(ix, phi, 4, psi.MORTON)
        assert st["leaf_cnt"].max() <= 2 * phi
    dels = synth.delete_ids(np.arange(60_000, dtype=np.uint32), 45_000, seed=82)
    for part in np.array_split(dels, 5):
        assert int(psi.to_u64(ix.batch_delete(part))[0]) == ref.batch_delete(part)
        ix.sync()
        check(ix, phi, 4, psi.MORTON)
    for a, b in zip(ix.export(), ref.dump()):
        np.testing.assert_array_equal(a, b)
