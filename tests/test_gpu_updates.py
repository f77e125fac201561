"""GPU parity of batch insert and batch delete against the oracle.

After every update: the sorted dump (keys, ids, coordinates) equals the
oracle's set bit for bit, the structure satisfies the invariants in
invariants.py, and kNN / range results equal the oracle's.
"""
import sys

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


def bits_of(dim):
    return 30 if dim == 2 else 21


class Pair:
    def __init__(self, psi, dim, curve, phi=32, B=8):
        self.psi = psi
        self.dim, self.curve, self.phi, self.B = dim, curve, phi, B
        self.g = psi.Index(dim, curve, phi, B)
        self.r = oracle.RefIndex(dim, curve, phi, B)

    def build(self, pts):
        self.g.build(pts)
        self.r.build(pts)

    def insert(self, pts):
        gi = self.psi.to_u32(self.g.batch_insert(pts))
        ri = self.r.batch_insert(pts)
        np.testing.assert_array_equal(gi, ri)

    def delete(self, ids):
        gd = int(self.psi.to_u64(self.g.batch_delete(ids))[0])
        rd = self.r.batch_delete(ids)
        assert gd == rd, (gd, rd)

    def verify(self, queries=None, k=10, boxes=None):
        self.g.sync()
        assert self.g.size() == self.r.size()
        assert self.g.next_id() == self.r.next_id()
        for a, b in zip(self.g.export(), self.r.dump()):
            np.testing.assert_array_equal(a, b)
        check(self.g, self.phi, self.B, self.curve)
        if queries is not None:
            ids, d2 = self.g.knn(queries, k)
            eids, ed2 = self.r.knn(queries, k)
            np.testing.assert_array_equal(self.psi.to_u64(d2), ed2)
            np.testing.assert_array_equal(self.psi.to_u32(ids), eids)
        if boxes is not None:
            np.testing.assert_array_equal(self.psi.to_u64(self.g.range_count(boxes)), self.r.range_count(boxes))


@pytest.mark.parametrize("dim,curve", [(2, 0), (2, 1), (3, 1)])
@pytest.mark.parametrize("dist", ["uniform", "varden"])
def test_insert_parity(psi, dim, curve, dist):
    say(f"insert dim={dim} curve={curve} dist={dist}")
    bits = bits_of(dim)
    data, ins, q = synth.workload(dist, dim, bits, seed=11, n=50_000, n_insert=30_000, n_query=500)
    P = Pair(psi, dim, curve)
    P.build(data)
    P.insert(ins[:100])        # tiny batch: appends only
    P.verify()
    P.insert(ins[100:30_000])  # large batch: splits
    P.verify(q, 10, synth.boxes(q[:200], bits, seed=12))


@pytest.mark.parametrize("dim,curve", [(2, 1), (3, 0), (3, 1)])
@pytest.mark.parametrize("dist", ["uniform", "varden"])
def test_delete_parity(psi, dim, curve, dist):
    say(f"delete dim={dim} curve={curve} dist={dist}")
    bits = bits_of(dim)
    data, _, q = synth.workload(dist, dim, bits, seed=13, n=60_000, n_query=400)
    P = Pair(psi, dim, curve)
    P.build(data)
    dels = synth.delete_ids(np.arange(60_000, dtype=np.uint32), 20_000, seed=14)
    P.delete(dels[:50])
    P.verify()
    junk = np.array([59_999, 70_000, 0xFFFFFFFE, dels[3], dels[3]], np.uint32)  # repeats, unknown, dead
    P.delete(np.concatenate([dels[50:], junk]))
    P.verify(q, 16, synth.boxes(q[:200], bits, seed=15))


def test_delete_contiguous_region(psi):
    # removing every point of a key range empties runs of consecutive leaves,
    # which must be regrouped with their neighbours
    say("delete region")
    P = Pair(psi, 2, 1)
    data = synth.uniform(80_000, 2, 30, seed=21)
    P.build(data)
    k, i, _ = P.r.dump()
    P.delete(i[10_000:35_000])
    P.verify(synth.uniform(300, 2, 30, seed=22, purpose=synth.P_QUERY), 12)
    P.delete(i[:9_990])  # leaves a handful of points at the front
    P.verify()


def test_delete_everything_then_insert(psi):
    say("delete all")
    P = Pair(psi, 3, 1, phi=8, B=4)
    data = synth.uniform(5_000, 3, 21, seed=31)
    P.build(data)
    P.delete(np.arange(5_000, dtype=np.uint32))
    P.verify()
    assert P.g.size() == 0
    P.delete(np.arange(10, dtype=np.uint32))  # nothing left to delete
    P.insert(synth.uniform(700, 3, 21, seed=32))
    P.verify(synth.uniform(50, 3, 21, seed=33, purpose=synth.P_QUERY), 5)


def test_insert_into_empty(psi):
    say("insert into empty")
    P = Pair(psi, 2, 0)
    P.build(np.zeros((0, 2), np.uint32))
    P.insert(synth.uniform(1_000, 2, 30, seed=41))
    P.verify()
    P.insert(synth.uniform(3_000, 2, 30, seed=42))
    P.verify(synth.uniform(100, 2, 30, seed=43, purpose=synth.P_QUERY), 7)


def test_insert_then_delete_restores(psi):
    say("insert then delete restores")
    P = Pair(psi, 3, 1)
    data = synth.uniform(40_000, 3, 21, seed=51)
    P.build(data)
    before = P.g.export()
    extra = synth.varden(25_000, 3, 21, seed=52)
    P.insert(extra)
    P.delete(np.arange(40_000, 65_000, dtype=np.uint32)[::-1].copy())
    P.verify()
    for a, b in zip(before, P.g.export()):
        np.testing.assert_array_equal(a, b)


def test_duplicate_points(psi):
    say("duplicates")
    P = Pair(psi, 2, 1, phi=4, B=2)
    base = synth.uniform(2_000, 2, 3, seed=61)  # 64 distinct points
    P.build(base)
    P.insert(synth.uniform(3_000, 2, 3, seed=62))
    P.verify(synth.uniform(100, 2, 3, seed=63, purpose=synth.P_QUERY), 20)
    P.delete(synth.delete_ids(np.arange(5_000, dtype=np.uint32), 2_500, seed=64))
    P.verify(synth.uniform(100, 2, 3, seed=65, purpose=synth.P_QUERY), 20)


@pytest.mark.parametrize("rounds", [6])
def test_incremental_mix(psi, rounds):
    # the paper's incremental workload in miniature: many batches of inserts
    # and deletes, checked after each one
    say("incremental mix")
    P = Pair(psi, 2, 1, phi=16, B=4)
    P.build(synth.varden(20_000, 2, 30, seed=71))
    live = np.arange(20_000, dtype=np.uint32)
    for r in range(rounds):
        ins = synth.varden(7_000, 2, 30, seed=100 + r)
        nid = P.r.next_id()
        P.insert(ins)
        live = np.concatenate([live, np.arange(nid, nid + 7_000, dtype=np.uint32)])
        d = synth.delete_ids(live, 6_000, seed=200 + r)
        P.delete(d)
        live = np.setdiff1d(live, d)
        P.verify(synth.uniform(64, 2, 30, seed=300 + r, purpose=synth.P_QUERY), 9)


def test_small_config_end_to_end(psi):
    # SPaC-Z, 2D, 1e6 uniform points in [0, 2^30)^2 (seed 1), phi 32:
    # build, insert 1e5, delete 1e5 existing ids, 1e4 kNN queries (k = 10)
    say("1e6 end to end")
    data, ins, q = synth.workload("uniform", 2, 30, seed=1, n=1_000_000, n_insert=100_000, n_query=10_000)
    P = Pair(psi, 2, 0)
    P.build(data)
    P.insert(ins)
    P.delete(synth.delete_ids(np.arange(1_100_000, dtype=np.uint32), 100_000, seed=1))
    P.verify(q, 10)


@pytest.mark.parametrize("m", [10_240, 10_241, 16_384, 16_385])
def test_batch_sizes_at_the_one_launch_limits(psi, m):
    """Batches at the limits of the one-workgroup sort (10240 pairs) and scan
    (16384 words), on both sides, with random delete order and repeats."""
    say(f"batch limits m={m}")
    data, ins, q = synth.workload("uniform", 3, 21, seed=91, n=60_000, n_insert=m, n_query=300)
    P = Pair(psi, 3, 1)
    P.build(data)
    P.insert(ins)
    P.verify(queries=q)
    live = np.arange(P.r.next_id(), dtype=np.uint32)
    dels = synth.delete_ids(live, m - 5, seed=92)
    dels = np.concatenate([dels, dels[:5]])  # five repeated ids: m in all
    P.delete(dels[np.argsort(synth.draws(synth.stream_key(93, synth.P_AUX), 0, m), kind="stable")])
    P.verify(queries=q)
