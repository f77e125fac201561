"""Parity at the full configuration sizes (1e8 points), in the launch
configuration bench.py times.

The oracle cannot rebuild 1e8 points in a test's time, so the checks are:
  * build: the sorted dump is strictly increasing in (key, id), its ids are a
    permutation of 0..n-1, every row's point equals the input point of its id,
    and the key of a seeded sample of rows equals the oracle's key; the leaf
    directory equals the closed-form chunking of the dump (sizes, pivots,
    exact boxes) and every node level is the union/sum of the one below;
  * updates: the dump is exactly the expected set (ids and points), still
    sorted, and the structure invariants hold;
  * queries: a seeded sample of kNN queries and boxes is brute-forced by the
    oracle over all points; every reported range id is checked to lie in its
    box and the report lengths equal the counts.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

N = 100_000_000


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


def lex_sorted(k, i):
    return bool(np.all((k[:-1] < k[1:]) | ((k[:-1] == k[1:]) & (i[:-1] < i[1:]))))


def check_directory(ix, keys, ids, pts, B):
    st = ix.structure()
    L, h = st["n_leaves"], st["height"]
    cnt = st["leaf_cnt"].astype(np.int64)
    assert cnt.sum() == len(ids)
    starts = np.concatenate(([0], np.cumsum(cnt)[:-1]))
    np.testing.assert_array_equal(st["piv_key"] <= keys[starts], True)
    np.testing.assert_array_equal(st["leaf_lo"], np.minimum.reduceat(pts, starts, axis=0))
    np.testing.assert_array_equal(st["leaf_hi"], np.maximum.reduceat(pts, starts, axis=0))
    sizes = st["level_sizes"]
    offs = np.concatenate(([0], np.cumsum(sizes)))
    lo, hi, c = st["node_lo"], st["node_hi"], st["node_cnt"].astype(np.int64)
    for lev in range(h):
        first = np.arange(0, sizes[lev + 1], B)
        sl = slice(offs[lev + 1], offs[lev + 2])
        np.testing.assert_array_equal(lo[offs[lev]:offs[lev + 1]], np.minimum.reduceat(lo[sl], first, axis=0))
        np.testing.assert_array_equal(hi[offs[lev]:offs[lev + 1]], np.maximum.reduceat(hi[sl], first, axis=0))
        np.testing.assert_array_equal(c[offs[lev]:offs[lev + 1]], np.add.reduceat(c[sl], first))
    assert c[0] == len(ids)
    return st, cnt, starts


@pytest.mark.parametrize("dim,curve,dist", [(3, 1, "uniform"), (2, 0, "varden"), (3, 1, "varden")])
def test_fullsize_build_update_query(psi, dim, curve, dist):
    bits = 30 if dim == 2 else 21
    B = 8
    say(f"fullsize {dim}D curve={curve} {dist}: generating")
    data, ins, q = synth.workload(dist, dim, bits, seed=1, n=N, n_insert=1_000_000, n_query=10_000_000)
    ix = psi.Index(dim, curve, 32, B)
    say("build")
    ix.build(data)
    ix.sync()
    keys, ids, pts = ix.export()
    assert lex_sorted(keys, ids)
    np.testing.assert_array_equal(np.sort(ids), np.arange(N, dtype=np.uint32))
    np.testing.assert_array_equal(pts, data[ids])
    rows = synth.sample_rows(N, 20_000, seed=2)
    np.testing.assert_array_equal(keys[rows], oracle.encode(pts[rows], dim, curve))
    st, cnt, starts = check_directory(ix, keys, ids, pts, B)
    L = -(-N // 32)
    assert st["n_leaves"] == L
    b = (np.arange(L + 1, dtype=np.int64) * N) // L  # closed-form chunking
    np.testing.assert_array_equal(cnt, np.diff(b))
    np.testing.assert_array_equal(st["piv_key"], keys[b[:-1]])
    np.testing.assert_array_equal(st["piv_id"], ids[b[:-1]])
    del keys, pts

    say("queries")
    for k in (1, 10, 100):
        kid, kd2 = ix.knn(q, k)
        sample = synth.sample_rows(len(q), 64, seed=k)
        eid, ed2 = oracle.knn_points(data, q[sample], k)
        np.testing.assert_array_equal(psi.to_u64(kd2)[sample], ed2)
        np.testing.assert_array_equal(psi.to_u32(kid)[sample], eid)
        del kid, kd2
    bx = synth.boxes(q[:1_000_000], bits, seed=3)
    cnts = psi.to_u64(ix.range_count(bx))
    sample = synth.sample_rows(len(bx), 64, seed=4)
    np.testing.assert_array_equal(cnts[sample], oracle.range_count_points(data, bx[sample]))
    off, rid = ix.range_report(bx, ix.range_count(bx))
    off, rid = psi.to_u64(off), psi.to_u32(rid)
    np.testing.assert_array_equal(np.diff(off), cnts)
    for s in sample[:16]:
        got = rid[off[s]:off[s + 1]]
        assert np.unique(got).size == got.size
        p = data[got]
        assert np.all((p >= bx[s, 0]) & (p <= bx[s, 1]))
    del rid

    say("updates")
    new_ids = psi.to_u32(ix.batch_insert(ins))
    np.testing.assert_array_equal(new_ids, np.arange(N, N + len(ins), dtype=np.uint32))
    dels = synth.delete_ids(np.arange(N + len(ins), dtype=np.uint32), 1_000_000, seed=5)
    nd = int(psi.to_u64(ix.batch_delete(dels))[0])
    assert nd == len(dels)
    ix.sync()
    keys, ids, pts = ix.export()
    allp = np.concatenate([data, ins])
    keep = np.ones(N + len(ins), bool)
    keep[dels] = False
    np.testing.assert_array_equal(np.sort(ids), np.nonzero(keep)[0].astype(np.uint32))
    assert lex_sorted(keys, ids)
    np.testing.assert_array_equal(pts, allp[ids])
    rows = synth.sample_rows(len(ids), 20_000, seed=6)
    np.testing.assert_array_equal(keys[rows], oracle.encode(pts[rows], dim, curve))
    st = ix.structure()
    c = st["leaf_cnt"].astype(np.int64)
    assert c.min() >= 16 and c.max() <= 64
    lids, lpts = ix.leaves()
    starts = np.concatenate(([0], np.cumsum(c)[:-1]))
    np.testing.assert_array_equal(st["leaf_lo"], np.minimum.reduceat(lpts, starts, axis=0))
    np.testing.assert_array_equal(st["leaf_hi"], np.maximum.reduceat(lpts, starts, axis=0))
    # every leaf holds exactly the next run of the sorted dump (as a set)
    owner = np.repeat(np.arange(len(c)), c)
    pos = np.empty(N + len(ins), np.int64)
    pos[ids] = np.arange(len(ids))
    lp = pos[lids]
    assert np.all(np.minimum.reduceat(lp, starts) == starts)
    assert np.all(np.maximum.reduceat(lp, starts) == starts + c - 1)
    del owner
    kid, kd2 = ix.knn(q, 10)
    sample = synth.sample_rows(len(q), 64, seed=7)
    eid, ed2 = oracle.knn_points(allp[keep], q[sample], 10)
    live = np.nonzero(keep)[0].astype(np.uint32)
    np.testing.assert_array_equal(psi.to_u64(kd2)[sample], ed2)
    np.testing.assert_array_equal(psi.to_u32(kid)[sample], live[eid])
    say("done")
