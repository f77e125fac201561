"""Parity at the full configuration sizes (1e8 points), in the launch
configuration bench.py times.

The oracle cannot rebuild 1e8 points in a test's time, so the checks are:
  * build: the sorted dump is strictly increasing in (key, id), its ids are a
    permutation of 0..n-1, every row's point equals the input point of its id,
    and the key of a seeded sample of rows equals the oracle's key; the leaf
    directory equals the closed-form chunking of the dump (sizes, pivots,
    exact boxes) and every node level is the union/sum of the one below;
  * updates: the dump is exactly the expected set (ids and points), still
    sorted; every leaf holds the next run of the dump, pivots bracket it,
    leaf boxes are tight and every node level is again the union/sum of the
    one below;
  * queries: a seeded sample of kNN queries and boxes is brute-forced by the
    oracle over all points; every one of the kNN rows is checked for what
    holds at any size (ascending in (d2, id), d2 equal to the squared
    distance to the returned point, which makes the ids distinct), and every
    reported id for lying in its box, once per box, with report lengths equal
    to the counts. Those all-row checks run as plain torch tensor arithmetic
    on the device: they recompute properties, not the index.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

N = 100_000_000
THREADS = 16  # oracle brute-force threads (the host share of one GPU)


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


def check_levels(st, B):
    """Every node level is the union (boxes) and sum (counts) of the one below."""
    h = st["height"]
    sizes = st["level_sizes"]
    offs = np.concatenate(([0], np.cumsum(sizes)))
    lo, hi, c = st["node_lo"], st["node_hi"], st["node_cnt"].astype(np.int64)
    np.testing.assert_array_equal(lo[offs[h]:offs[h + 1]], st["leaf_lo"])
    np.testing.assert_array_equal(hi[offs[h]:offs[h + 1]], st["leaf_hi"])
    np.testing.assert_array_equal(c[offs[h]:offs[h + 1]], st["leaf_cnt"])
    for lev in range(h):
        first = np.arange(0, sizes[lev + 1], B)
        sl = slice(offs[lev + 1], offs[lev + 2])
        np.testing.assert_array_equal(lo[offs[lev]:offs[lev + 1]], np.minimum.reduceat(lo[sl], first, axis=0))
        np.testing.assert_array_equal(hi[offs[lev]:offs[lev + 1]], np.maximum.reduceat(hi[sl], first, axis=0))
        np.testing.assert_array_equal(c[offs[lev]:offs[lev + 1]], np.add.reduceat(c[sl], first))
    return c[0]


def check_directory(ix, keys, ids, pts, B):
    st = ix.structure()
    cnt = st["leaf_cnt"].astype(np.int64)
    assert cnt.sum() == len(ids)
    starts = np.concatenate(([0], np.cumsum(cnt)[:-1]))
    np.testing.assert_array_equal(st["piv_key"] <= keys[starts], True)
    np.testing.assert_array_equal(st["leaf_lo"], np.minimum.reduceat(pts, starts, axis=0))
    np.testing.assert_array_equal(st["leaf_hi"], np.maximum.reduceat(pts, starts, axis=0))
    assert check_levels(st, B) == len(ids)
    return st, cnt, starts


def check_after_updates(psi, ix, allp, keep, dim, curve, phi, B):
    """The dump is exactly the live set; every leaf holds the next run of it;
    pivots bracket their runs; leaf boxes are tight; node levels are the
    union/sum of the level below."""
    keys, ids, pts = ix.export()
    np.testing.assert_array_equal(np.sort(ids), np.nonzero(keep)[0].astype(np.uint32))
    assert lex_sorted(keys, ids)
    np.testing.assert_array_equal(pts, allp[ids])
    rows = synth.sample_rows(len(ids), 20_000, seed=6)
    np.testing.assert_array_equal(keys[rows], oracle.encode(pts[rows], dim, curve))
    st = ix.structure()
    c = st["leaf_cnt"].astype(np.int64)
    assert c.sum() == len(ids)
    assert c.min() >= (phi + 1) // 2 and c.max() <= 2 * phi, (c.min(), c.max())
    lids, lpts = ix.leaves()
    starts = np.concatenate(([0], np.cumsum(c)[:-1]))
    np.testing.assert_array_equal(st["leaf_lo"], np.minimum.reduceat(lpts, starts, axis=0))
    np.testing.assert_array_equal(st["leaf_hi"], np.maximum.reduceat(lpts, starts, axis=0))
    pos = np.empty(len(allp), np.int64)
    pos[ids] = np.arange(len(ids))
    lp = pos[lids]
    del lids, lpts
    assert np.all(np.minimum.reduceat(lp, starts) == starts)
    assert np.all(np.maximum.reduceat(lp, starts) == starts + c - 1)
    del lp, pos
    # pivot j <= the first entry of run j, and > the last entry of run j - 1
    pk, pi = st["piv_key"], st["piv_id"]
    fk, fi = keys[starts], ids[starts]
    assert np.all((pk < fk) | ((pk == fk) & (pi <= fi)))
    lk, li = keys[starts[1:] - 1], ids[starts[1:] - 1]
    assert np.all((pk[1:] > lk) | ((pk[1:] == lk) & (pi[1:] > li)))
    assert check_levels(st, B) == len(ids)


def knn_rows_check(torch, pts_d, q_d, kid, kd2, live_d=None):
    """Every row: real ids (of live points), d2 equal to the squared distance
    from the query to the returned point, ascending in (d2, id) (so the ids
    of a row are distinct)."""
    n, k = kid.shape
    ch = max(1, 20_000_000 // k)
    for a in range(0, n, ch):
        ids = kid[a:a + ch].long()
        d2 = kd2[a:a + ch]
        assert bool((ids >= 0).all()), "padding in a full-size kNN row"
        if live_d is not None:
            assert bool(live_d[ids].all()), "a returned id is not live"
        p = pts_d[ids]
        dd = ((p - q_d[a:a + ch].unsqueeze(1)) ** 2).sum(-1)
        bad = (dd != d2).any(1).nonzero()
        assert bad.numel() == 0, f"row {a + int(bad[0])}: d2 differs from the returned point's distance"
        if k > 1:
            ok = (d2[:, :-1] < d2[:, 1:]) | ((d2[:, :-1] == d2[:, 1:]) & (ids[:, :-1] < ids[:, 1:]))
            assert bool(ok.all()), "a kNN row is not ascending in (d2, id)"


def report_rows_check(torch, pts_d, bx_d, off, rid, cnt):
    """Report lengths equal the counts; every reported id lies in its box and
    appears once per box."""
    assert torch.equal(off[1:] - off[:-1], cnt)
    nb = cnt.numel()
    off_h = off.cpu().numpy()
    bounds = [0]
    while bounds[-1] < nb:  # chunks of about 2e7 ids (a single box may exceed it)
        b0 = bounds[-1]
        b1 = int(np.searchsorted(off_h, off_h[b0] + 20_000_000, side="right")) - 1
        bounds.append(min(nb, max(b1, b0 + 1)))
    for b0, b1 in zip(bounds[:-1], bounds[1:]):
        o0, o1 = int(off_h[b0]), int(off_h[b1])
        if o1 == o0:
            continue
        ids = rid[o0:o1].long()
        box_of = torch.repeat_interleave(torch.arange(b0, b1, device=ids.device), cnt[b0:b1])
        p = pts_d[ids]
        inside = (p >= bx_d[box_of, 0]) & (p <= bx_d[box_of, 1])
        assert bool(inside.all()), "a reported id lies outside its box"
        s, _ = torch.sort(box_of * (1 << 32) + ids)
        assert bool((s[1:] != s[:-1]).all()), "an id reported twice for one box"


def sampled_queries(psi, ix, data, q, bx, ks, samples, live=None, pts_d=None, q_d=None, torch=None):
    """kNN for every k and range counts/reports: sampled rows against the
    oracle's brute force, every row against the properties above."""
    bx_d = torch.from_numpy(bx.astype(np.int64)).to(pts_d.device)
    for k in ks:
        kid, kd2 = ix.knn(q, k)
        knn_rows_check(torch, pts_d, q_d, kid, kd2)
        rows = synth.sample_rows(len(q), samples.get(k, 64), seed=k)
        eid, ed2 = oracle.knn_points(data, q[rows], k, threads=THREADS)
        got_id, got_d2 = psi.to_u32(kid[torch.from_numpy(rows).to(kid.device)]), psi.to_u64(kd2[torch.from_numpy(rows).to(kd2.device)])
        np.testing.assert_array_equal(got_d2, ed2)
        np.testing.assert_array_equal(got_id, eid if live is None else live[eid])
        del kid, kd2
    cnt = ix.range_count(bx)
    rows = synth.sample_rows(len(bx), samples.get("range", 512), seed=4)
    np.testing.assert_array_equal(psi.to_u64(cnt)[rows], oracle.range_count_points(data, bx[rows], threads=THREADS))
    off, rid = ix.range_report(bx, cnt)
    report_rows_check(torch, pts_d, bx_d, off, rid, cnt)
    say(f"  report rows: {int(off[-1])} ids over {len(bx)} boxes")


def box_sides(dim, dist):
    # 3D: the bench's boxes; 2D: sides that hold hundreds of points on
    # average (Varden's clusters are dense: smaller boxes)
    if dim == 2:
        return dict(side_lo=15, side_hi=23) if dist == "uniform" else dict(side_lo=6, side_hi=14)
    return dict(side_lo=8, side_hi=18)


def build_and_check(psi, dim, curve, dist, B, n_insert=1_000_000, nq=10_000_000):
    bits = 30 if dim == 2 else 21
    say(f"fullsize {dim}D curve={curve} {dist}: generating")
    data, ins, q = synth.workload(dist, dim, bits, seed=1, n=N, n_insert=n_insert, n_query=nq)
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
    return bits, data, ins, q, ix


@pytest.mark.parametrize("dim,curve,dist", [(3, 1, "uniform"), (2, 0, "varden"), (3, 1, "varden")])
def test_fullsize_build_update_query(psi, dim, curve, dist):
    import torch
    B = 8
    bits, data, ins, q, ix = build_and_check(psi, dim, curve, dist, B)
    dev = ix.device
    pts_d = torch.from_numpy(data.astype(np.int64)).to(dev)
    q_d = torch.from_numpy(q.astype(np.int64)).to(dev)
    say("queries")
    bx = synth.boxes(q[:1_000_000], bits, seed=3, **box_sides(dim, dist))
    sampled_queries(psi, ix, data, q, bx, (1, 10, 100), {1: 128, 10: 512, 100: 64, "range": 512},
                    pts_d=pts_d, q_d=q_d, torch=torch)
    del pts_d

    say("updates")
    new_ids = psi.to_u32(ix.batch_insert(ins))
    np.testing.assert_array_equal(new_ids, np.arange(N, N + len(ins), dtype=np.uint32))
    dels = synth.delete_ids(np.arange(N + len(ins), dtype=np.uint32), 1_000_000, seed=5)
    nd = int(psi.to_u64(ix.batch_delete(dels))[0])
    assert nd == len(dels)
    ix.sync()
    allp = np.concatenate([data, ins])
    keep = np.ones(N + len(ins), bool)
    keep[dels] = False
    check_after_updates(psi, ix, allp, keep, dim, curve, 32, B)
    kid, kd2 = ix.knn(q, 10)
    knn_rows_check(torch, torch.from_numpy(allp.astype(np.int64)).to(dev), q_d, kid, kd2,
                   live_d=torch.from_numpy(keep).to(dev))
    sample = synth.sample_rows(len(q), 128, seed=7)
    eid, ed2 = oracle.knn_points(allp[keep], q[sample], 10, threads=THREADS)
    live = np.nonzero(keep)[0].astype(np.uint32)
    np.testing.assert_array_equal(psi.to_u64(kd2)[sample], ed2)
    np.testing.assert_array_equal(psi.to_u32(kid)[sample], live[eid])
    say("done")


@pytest.mark.parametrize("curve,dist", [(1, "uniform"), (1, "varden"), (0, "uniform")])
def test_fullsize_2d_build_query(psi, curve, dist):
    """2D SPaC-H (uniform and Varden) and 2D SPaC-Z (uniform) at 1e8 points:
    the build against the closed form, 10-NN and range queries."""
    import torch
    B = 8
    nb = 100_000 if dist == "uniform" else 1_000_000
    bits, data, _, q, ix = build_and_check(psi, 2, curve, dist, B, n_insert=0, nq=10_000_000)
    dev = ix.device
    pts_d = torch.from_numpy(data.astype(np.int64)).to(dev)
    q_d = torch.from_numpy(q.astype(np.int64)).to(dev)
    say("queries")
    bx = synth.boxes(q[:nb], bits, seed=3, **box_sides(2, dist))
    sampled_queries(psi, ix, data, q, bx, (10,), {10: 256, "range": 256}, pts_d=pts_d, q_d=q_d, torch=torch)
    say("done")


def test_fullsize_large_batches(psi):
    """Insert 1e7 points into the 1e8-point 3D SPaC-H index, then delete 1e7
    ids drawn from all live ids (old and new): exact sets and the structure
    after each batch, then 10-NN queries on the result."""
    import torch
    B, dim, curve, m = 8, 3, 1, 10_000_000
    bits, data, ins, q, ix = build_and_check(psi, dim, curve, "uniform", B, n_insert=m, nq=1_000_000)
    dev = ix.device
    say("insert 1e7")
    new_ids = psi.to_u32(ix.batch_insert(ins))
    np.testing.assert_array_equal(new_ids, np.arange(N, N + m, dtype=np.uint32))
    ix.sync()
    allp = np.concatenate([data, ins])
    keep = np.ones(N + m, bool)
    check_after_updates(psi, ix, allp, keep, dim, curve, 32, B)
    say("delete 1e7")
    dels = synth.delete_ids(np.arange(N + m, dtype=np.uint32), m, seed=15)
    nd = int(psi.to_u64(ix.batch_delete(dels))[0])
    assert nd == m
    ix.sync()
    keep[dels] = False
    assert ix.size() == N
    check_after_updates(psi, ix, allp, keep, dim, curve, 32, B)
    say("queries")
    q_d = torch.from_numpy(q.astype(np.int64)).to(dev)
    kid, kd2 = ix.knn(q, 10)
    knn_rows_check(torch, torch.from_numpy(allp.astype(np.int64)).to(dev), q_d, kid, kd2,
                   live_d=torch.from_numpy(keep).to(dev))
    sample = synth.sample_rows(len(q), 256, seed=17)
    eid, ed2 = oracle.knn_points(allp[keep], q[sample], 10, threads=THREADS)
    live = np.nonzero(keep)[0].astype(np.uint32)
    np.testing.assert_array_equal(psi.to_u64(kd2)[sample], ed2)
    np.testing.assert_array_equal(psi.to_u32(kid)[sample], live[eid])
    bx = synth.boxes(q[:256], bits, seed=18)
    np.testing.assert_array_equal(psi.to_u64(ix.range_count(bx)),
                                  oracle.range_count_points(allp[keep], bx, threads=THREADS))
    say("done")
