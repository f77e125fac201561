"""Pins of the oracle's sort, canonical structure, updates and queries.

Each check uses something other than the oracle's own code: numpy's lexsort,
closed forms of the balanced chunking, brute-force numpy reductions, set
identities of insert/delete, hand-made lattices with known neighbours, and a
second brute force (full sort) for kNN.
"""
import numpy as np
import pytest

import synth


def _np_knn(pts, ids, q, k):
    """Independent numpy brute force: lexsort on (id, d2)."""
    out_i = np.full((len(q), k), 0xFFFFFFFF, np.uint32)
    out_d = np.full((len(q), k), 0xFFFFFFFFFFFFFFFF, np.uint64)
    P = pts.astype(np.int64)
    for r, qq in enumerate(q.astype(np.int64)):
        d2 = ((P - qq) ** 2).sum(axis=1).astype(np.uint64)
        o = np.lexsort((ids, d2))[:k]
        out_i[r, :len(o)] = ids[o]
        out_d[r, :len(o)] = d2[o]
    return out_i, out_d


def test_sort_pairs_against_numpy(ora):
    rng = np.random.default_rng(1)
    keys = rng.integers(0, 1000, size=20000, dtype=np.uint64)  # many equal keys
    ids = rng.permutation(20000).astype(np.uint32)
    k, i = ora.sort_pairs(keys, ids)
    o = np.lexsort((ids, keys))
    np.testing.assert_array_equal(k, keys[o])
    np.testing.assert_array_equal(i, ids[o])


@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 64, 65, 1000, 4097])
@pytest.mark.parametrize("dim,curve", [(2, 0), (2, 1), (3, 1)])
def test_canonical_structure_closed_form(ora, n, dim, curve):
    phi, B = 32, 4
    bits = 30 if dim == 2 else 21
    pts = synth.uniform(n, dim, bits, seed=n + 5)
    R = ora.RefIndex(dim, curve, phi, B)
    R.build(pts)
    keys, ids, dp = R.dump()
    st = R.structure()
    L = st["n_leaves"]
    assert L == (0 if n == 0 else -(-n // phi))
    if n == 0:
        return
    cnt = st["leaf_cnt"].astype(np.int64)
    assert cnt.sum() == n
    assert cnt.min() >= n // L and cnt.max() <= -(-n // L)
    if n >= phi:
        assert cnt.min() >= phi // 2 and cnt.max() <= phi
    starts = np.concatenate(([0], np.cumsum(cnt)[:-1]))
    np.testing.assert_array_equal(st["piv_key"], keys[starts])
    np.testing.assert_array_equal(st["piv_id"], ids[starts])
    np.testing.assert_array_equal(st["leaf_lo"], np.minimum.reduceat(dp, starts, axis=0))
    np.testing.assert_array_equal(st["leaf_hi"], np.maximum.reduceat(dp, starts, axis=0))
    # node levels: root first, leaves last; a parent is the union of its
    # (up to B) children one level down
    sizes = st["level_sizes"]
    h = st["height"]
    assert sizes[0] == 1 and sizes[h] == L
    assert B ** h >= L and (h == 0 or B ** (h - 1) < L)
    offs = np.concatenate(([0], np.cumsum(sizes)))
    lo, hi, c = st["node_lo"], st["node_hi"], st["node_cnt"]
    np.testing.assert_array_equal(lo[offs[h]:offs[h + 1]], st["leaf_lo"])
    np.testing.assert_array_equal(c[offs[h]:offs[h + 1]], cnt)
    for lev in range(h):
        child = np.arange(sizes[lev + 1])
        par = child // B
        clo, chi, cc = lo[offs[lev + 1]:offs[lev + 2]], hi[offs[lev + 1]:offs[lev + 2]], c[offs[lev + 1]:offs[lev + 2]]
        first = np.searchsorted(par, np.arange(sizes[lev]))
        np.testing.assert_array_equal(lo[offs[lev]:offs[lev + 1]], np.minimum.reduceat(clo, first, axis=0))
        np.testing.assert_array_equal(hi[offs[lev]:offs[lev + 1]], np.maximum.reduceat(chi, first, axis=0))
        np.testing.assert_array_equal(c[offs[lev]:offs[lev + 1]], np.add.reduceat(cc, first))
    assert c[0] == n


def test_two_leaf_split_sizes(ora):
    # n = phi + 1 gives two leaves of floor and ceil of (phi+1)/2
    R = ora.RefIndex(2, 0, 32, 2)
    R.build(synth.uniform(33, 2, 30, seed=1))
    np.testing.assert_array_equal(R.structure()["leaf_cnt"], [16, 17])


def test_build_sorted_and_ids(ora):
    pts = synth.uniform(3000, 3, 21, seed=2)
    R = ora.RefIndex(3, 1, 32, 8)
    R.build(pts)
    k, i, p = R.dump()
    assert np.all((k[:-1] < k[1:]) | ((k[:-1] == k[1:]) & (i[:-1] < i[1:])))
    np.testing.assert_array_equal(np.sort(i), np.arange(3000))
    np.testing.assert_array_equal(p, pts[i])
    np.testing.assert_array_equal(k, ora.encode(pts[i], 3, 1))


def test_out_of_range_rejected(ora):
    R = ora.RefIndex(3, 0, 32, 2)
    with pytest.raises(ValueError):
        R.build(np.array([[1 << 21, 0, 0]], np.uint32))
    R2 = ora.RefIndex(2, 0, 32, 2)
    with pytest.raises(ValueError):
        R2.build(np.array([[0, 1 << 31]], np.uint32))


@pytest.mark.parametrize("dim,curve", [(2, 0), (3, 1)])
def test_insert_into_empty_equals_build(ora, dim, curve):
    pts = synth.uniform(500, dim, 20, seed=3)
    A = ora.RefIndex(dim, curve)
    A.build(pts)
    B = ora.RefIndex(dim, curve)
    B.build(np.zeros((0, dim), np.uint32))
    ids = B.batch_insert(pts)
    np.testing.assert_array_equal(ids, np.arange(500))
    for a, b in zip(A.dump(), B.dump()):
        np.testing.assert_array_equal(a, b)


def test_insert_then_delete_restores(ora):
    pts = synth.uniform(2000, 2, 30, seed=4)
    extra = synth.uniform(700, 2, 30, seed=4, purpose=synth.P_INSERT)
    R = ora.RefIndex(2, 1)
    R.build(pts)
    before = R.dump()
    ids = R.batch_insert(extra)
    np.testing.assert_array_equal(ids, np.arange(2000, 2700))
    assert R.size() == 2700
    assert R.batch_delete(ids[::-1]) == 700
    for a, b in zip(before, R.dump()):
        np.testing.assert_array_equal(a, b)
    assert R.next_id() == 2700  # ids are never reused


def test_delete_set_semantics(ora):
    pts = synth.uniform(1000, 3, 21, seed=5)
    R = ora.RefIndex(3, 0)
    R.build(pts)
    batch = np.array([5, 5, 7, 999, 1000, 123456, 7, 0], np.uint32)  # repeats, unknown ids
    assert R.batch_delete(batch) == 4
    assert R.batch_delete(np.array([5, 0], np.uint32)) == 0  # already dead
    k, i, p = R.dump()
    assert set(i.tolist()) == set(range(1000)) - {0, 5, 7, 999}
    assert R.batch_delete(np.arange(1000, dtype=np.uint32)) == 996
    assert R.size() == 0


def test_duplicates_allowed(ora):
    R = ora.RefIndex(2, 1)
    R.build(np.array([[3, 4], [3, 4], [1, 1]], np.uint32))
    R.batch_insert(np.array([[3, 4]], np.uint32))
    k, i, p = R.dump()
    dup = np.isin(i, [0, 1, 3])
    assert (k[dup] == k[dup][0]).all()
    assert i[dup].tolist() == [0, 1, 3]  # equal keys ordered by id
    ids, d2 = R.knn(np.array([[3, 4]], np.uint32), 3)
    assert ids.tolist() == [[0, 1, 3]] and d2.tolist() == [[0, 0, 0]]


def test_knn_lattice_ties(ora):
    # 3x3 lattice, query at the centre: itself at 0, then four ties at 1
    # ordered by id, then four ties at 2 ordered by id
    g = np.array([[x, y] for y in range(10, 13) for x in range(20, 23)], np.uint32)
    perm = np.array([4, 7, 1, 8, 0, 2, 6, 3, 5])
    R = ora.RefIndex(2, 0, 4, 2)
    R.build(g[perm])
    ids, d2 = R.knn(np.array([[21, 11]], np.uint32), 9)
    pos = {tuple(g[perm][i]): i for i in range(9)}
    centre = pos[(21, 11)]
    ring1 = sorted(pos[p] for p in [(20, 11), (22, 11), (21, 10), (21, 12)])
    ring2 = sorted(pos[p] for p in [(20, 10), (22, 10), (20, 12), (22, 12)])
    assert ids[0].tolist() == [centre] + ring1 + ring2
    assert d2[0].tolist() == [0, 1, 1, 1, 1, 2, 2, 2, 2]
    # k cutting through a ring keeps its smallest ids, whatever the key order
    for k in range(1, 9):
        ids, d2 = R.knn(np.array([[21, 11]], np.uint32), k)
        assert ids[0].tolist() == ([centre] + ring1 + ring2)[:k], k


@pytest.mark.parametrize("dim", [2, 3])
def test_knn_ties_at_the_kth_distance(ora, dim):
    # a tiny domain: many equal points and equal distances, so the k-th
    # distance is shared by several points; the smallest ids among them win
    pts = synth.uniform(800, dim, 3, seed=7 + dim)
    q = synth.uniform(40, dim, 3, seed=8 + dim, purpose=synth.P_QUERY)
    R = ora.RefIndex(dim, 1)
    R.build(pts)
    for k in (3, 10, 33):
        a = R.knn(q, k)
        c = _np_knn(pts, np.arange(len(pts), dtype=np.uint32), q, k)
        np.testing.assert_array_equal(a[0], c[0])
        np.testing.assert_array_equal(a[1], c[1])


def test_knn_padding_when_k_exceeds_n(ora):
    R = ora.RefIndex(3, 1)
    R.build(np.array([[1, 2, 3], [4, 5, 6]], np.uint32))
    ids, d2 = R.knn(np.array([[0, 0, 0]], np.uint32), 4)
    assert ids[0].tolist() == [0, 1, 0xFFFFFFFF, 0xFFFFFFFF]
    assert d2[0].tolist() == [14, 77, 2**64 - 1, 2**64 - 1]
    E = ora.RefIndex(2, 0)
    E.build(np.zeros((0, 2), np.uint32))
    ids, d2 = E.knn(np.array([[1, 1]], np.uint32), 2)
    assert ids.tolist() == [[0xFFFFFFFF] * 2]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("k", [1, 5, 16, 40])
def test_knn_two_brute_forces_agree(ora, dim, k):
    bits = 10  # small domain: many exact distance ties
    pts = synth.uniform(1500, dim, bits, seed=k + dim)
    q = synth.uniform(60, dim, bits, seed=k + dim, purpose=synth.P_QUERY)
    R = ora.RefIndex(dim, 1)
    R.build(pts)
    a = R.knn(q, k)
    b = R.knn_fullsort(q, k)
    c = _np_knn(pts, np.arange(len(pts), dtype=np.uint32), q, k)
    for x, y, z in zip(a, b, c):
        np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(x, z)


def test_knn_full_width_2d_distances(ora):
    # 2D coordinates up to 2^31-1: squared distances up to ~2^63 stay exact
    pts = np.array([[0, 0], [2**31 - 1, 2**31 - 1], [2**31 - 1, 0]], np.uint32)
    R = ora.RefIndex(2, 1)
    R.build(pts)
    ids, d2 = R.knn(np.array([[0, 0]], np.uint32), 3)
    m = 2**31 - 1
    assert ids[0].tolist() == [0, 2, 1]
    assert d2[0].tolist() == [0, m * m, 2 * m * m]


@pytest.mark.parametrize("dim", [2, 3])
def test_range_invariants(ora, dim):
    bits = 16
    pts = synth.uniform(3000, dim, bits, seed=21)
    R = ora.RefIndex(dim, 0)
    R.build(pts)
    full = np.zeros((1, 2, dim), np.uint32)
    full[0, 1, :] = (1 << bits) - 1
    assert R.range_count(full)[0] == 3000
    bx = synth.boxes(synth.uniform(200, dim, bits, seed=22), bits, seed=23, side_lo=6, side_hi=14)
    cnt = R.range_count(bx)
    ref = np.array([np.all((pts >= b[0]) & (pts <= b[1]), axis=1).sum() for b in bx])
    np.testing.assert_array_equal(cnt, ref)
    # additivity over a split along axis 0
    mid = ((bx[:, 0, 0].astype(np.int64) + bx[:, 1, 0]) // 2).astype(np.uint32)
    left, right = bx.copy(), bx.copy()
    left[:, 1, 0] = mid
    right[:, 0, 0] = mid + 1
    np.testing.assert_array_equal(R.range_count(left) + R.range_count(right), cnt)
    off, ids = R.range_report(bx)
    np.testing.assert_array_equal(np.diff(off), cnt)
    for b in range(0, 200, 17):
        exp = np.nonzero(np.all((pts >= bx[b, 0]) & (pts <= bx[b, 1]), axis=1))[0]
        np.testing.assert_array_equal(ids[off[b]:off[b + 1]], exp)
    empty = bx[:3].copy()
    empty[:, 0, dim - 1] = empty[:, 1, dim - 1] + 1
    assert R.range_count(empty).tolist() == [0, 0, 0]


@pytest.mark.parametrize("dist", ["sweepline", "varden"])
def test_incremental_batches_equal_one_build(ora, dist):
    """Building from empty by many insertion batches gives the set (keys, ids,
    points) of one build of all points, and deleting in batches empties it
    (the paper's incremental workload, Sec. 5.1, on the oracle)."""
    pts = synth.points(dist, 6000, 2, 30, seed=71)
    inc = ora.RefIndex(2, 1, 8, 4)
    inc.build(np.zeros((0, 2), np.uint32))
    for i in range(0, 6000, 250):
        np.testing.assert_array_equal(inc.batch_insert(pts[i:i + 250]), np.arange(i, i + 250, dtype=np.uint32))
    one = ora.RefIndex(2, 1, 8, 4)
    one.build(pts)
    for a, b in zip(inc.dump(), one.dump()):
        np.testing.assert_array_equal(a, b)
    for i in range(0, 6000, 250):
        assert inc.batch_delete(np.arange(i, i + 250, dtype=np.uint32)) == 250
    assert inc.size() == 0
