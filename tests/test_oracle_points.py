"""Pins of the oracle's raw-point brute forces (knn_points, range_count_points).

These two functions check the largest GPU configurations (sampled queries over
1e8 points, the P-Orth tree's queries, many indexes), so they are pinned by
things other than their own code: a numpy lexsort on (d2, id) over the same
points, the oracle's set index (RefIndex) built from the same rows (its ids
are the row numbers too), hand lattices whose neighbours are known, a closed
form for the full domain and for boxes cut at single points, and a plain
numpy scan for counts. kNN is defined in Sec. 2.2 (k nearest by Euclidean
distance; ties by the smaller id, padding past n); range count is the number
of points inside a closed axis-aligned box (Sec. 2.2).
"""
import numpy as np
import pytest

import synth

PAD_ID = 0xFFFFFFFF
PAD_D2 = 0xFFFFFFFFFFFFFFFF


def _np_knn(pts, q, k):
    n = len(pts)
    out_i = np.full((len(q), k), PAD_ID, np.uint32)
    out_d = np.full((len(q), k), PAD_D2, np.uint64)
    P = pts.astype(np.int64)
    ids = np.arange(n, dtype=np.uint32)
    for r, qq in enumerate(q.astype(np.int64)):
        d2 = ((P - qq) ** 2).sum(axis=1).astype(np.uint64)
        o = np.lexsort((ids, d2))[:k]
        out_i[r, :len(o)] = ids[o]
        out_d[r, :len(o)] = d2[o]
    return out_i, out_d


def _np_count(pts, boxes):
    b = boxes.reshape(len(boxes), 2, -1).astype(np.int64)
    P = pts.astype(np.int64)
    return np.array([int(np.all((P >= lo) & (P <= hi), axis=1).sum()) for lo, hi in b], np.uint64)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("k", [1, 4, 10, 33])
def test_knn_points_tiny_domain_ties(ora, dim, k):
    # coordinates in [0, 4): hundreds of equal points, so the k-th distance is
    # shared by many of them; only the smallest ids may be kept
    pts = synth.uniform(600, dim, 2, seed=31 + dim)
    q = synth.uniform(50, dim, 2, seed=32 + dim, purpose=synth.P_QUERY)
    a = ora.knn_points(pts, q, k)
    c = _np_knn(pts, q, k)
    np.testing.assert_array_equal(a[0], c[0])
    np.testing.assert_array_equal(a[1], c[1])


@pytest.mark.parametrize("dim,curve", [(2, 0), (3, 1)])
def test_knn_points_equals_set_index(ora, dim, curve):
    # the set index keeps its points in key order, the raw scan in id order:
    # the two walk the points differently and must still agree
    pts = synth.uniform(3000, dim, 6, seed=41)
    q = synth.uniform(80, dim, 6, seed=42, purpose=synth.P_QUERY)
    R = ora.RefIndex(dim, curve)
    R.build(pts)
    for k in (1, 7, 50):
        a = ora.knn_points(pts, q, k)
        b = R.knn(q, k)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


def test_knn_points_lattice_ring_order(ora):
    # 3x3 lattice around (21, 11) with ids out of spatial order: the centre,
    # then the four points at distance 1 by id, then the four corners by id;
    # every k that cuts a ring keeps that ring's smallest ids
    g = np.array([[x, y] for y in range(10, 13) for x in range(20, 23)], np.uint32)
    perm = np.array([8, 3, 5, 0, 4, 7, 1, 6, 2])
    pts = g[perm]
    pos = {tuple(int(v) for v in pts[i]): i for i in range(9)}
    centre = pos[(21, 11)]
    ring1 = sorted(pos[p] for p in [(20, 11), (22, 11), (21, 10), (21, 12)])
    ring2 = sorted(pos[p] for p in [(20, 10), (22, 10), (20, 12), (22, 12)])
    want = [centre] + ring1 + ring2
    for k in range(1, 10):
        ids, d2 = ora.knn_points(pts, np.array([[21, 11]], np.uint32), k)
        assert ids[0].tolist() == want[:k], k
        assert d2[0].tolist() == [0, 1, 1, 1, 1, 2, 2, 2, 2][:k], k


def test_knn_points_padding_and_equal_points(ora):
    # k > n pads; equal points come back in id order at the same distance
    pts = np.array([[5, 5, 5], [5, 5, 5], [0, 0, 0], [5, 5, 5]], np.uint32)
    ids, d2 = ora.knn_points(pts, np.array([[5, 5, 6]], np.uint32), 6)
    assert ids[0].tolist() == [0, 1, 3, 2, PAD_ID, PAD_ID]
    assert d2[0].tolist() == [1, 1, 1, 25 + 25 + 36, PAD_D2, PAD_D2]
    ids, d2 = ora.knn_points(np.zeros((0, 2), np.uint32), np.array([[1, 1]], np.uint32), 2)
    assert ids.tolist() == [[PAD_ID, PAD_ID]]
    assert d2.tolist() == [[PAD_D2, PAD_D2]]


def test_knn_points_full_width_2d(ora):
    m = 2**31 - 1
    pts = np.array([[m, m], [m, 0], [0, 0]], np.uint32)
    ids, d2 = ora.knn_points(pts, np.array([[0, 0]], np.uint32), 3)
    assert ids[0].tolist() == [2, 1, 0]
    assert d2[0].tolist() == [0, m * m, 2 * m * m]


def test_knn_points_threads_do_not_change_results(ora):
    pts = synth.uniform(2000, 3, 4, seed=51)
    q = synth.uniform(64, 3, 4, seed=52, purpose=synth.P_QUERY)
    a = ora.knn_points(pts, q, 12, threads=1)
    b = ora.knn_points(pts, q, 12, threads=8)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("dim", [2, 3])
def test_range_count_points_against_numpy_and_set_index(ora, dim):
    pts = synth.uniform(2500, dim, 8, seed=61 + dim)
    centres = synth.uniform(300, dim, 8, seed=62, purpose=synth.P_QUERY)
    boxes = synth.boxes(centres, 8, seed=62, side_lo=0, side_hi=7)
    a = ora.range_count_points(pts, boxes)
    np.testing.assert_array_equal(a, _np_count(pts, boxes))
    R = ora.RefIndex(dim, 0)
    R.build(pts)
    np.testing.assert_array_equal(a, R.range_count(boxes))


@pytest.mark.parametrize("dim", [2, 3])
def test_range_count_points_closed_boxes(ora, dim):
    # a box of one grid point holds exactly the points equal to it (the first
    # row included), a box whose upper face passes through a point holds it,
    # the full domain holds all, and lo > hi in any axis holds none
    rng = np.random.default_rng(70 + dim)
    pts = rng.integers(0, 6, size=(200, dim), dtype=np.uint32)
    top = (1 << 31) - 1 if dim == 2 else (1 << 21) - 1
    single = [np.concatenate([p, p]) for p in pts[:40]]
    full = np.array([0] * dim + [top] * dim, np.uint32)
    face = np.concatenate([np.zeros(dim, np.uint32), pts[0]])
    empty = np.array([3] * dim + [2] + [5] * (dim - 1), np.uint32)
    boxes = np.array(single + [full, face, empty], np.uint32)
    got = ora.range_count_points(pts, boxes)
    for b in range(40):
        assert got[b] == int(np.all(pts == pts[b], axis=1).sum()), b
    assert got[40] == len(pts)
    assert got[41] == int(np.all(pts <= pts[0], axis=1).sum())
    assert got[42] == 0
    # additivity over a split of the domain along axis 0
    cut = 2
    lo_half = np.array([0] * dim + [cut] + [top] * (dim - 1), np.uint32)
    hi_half = np.array([cut + 1] + [0] * (dim - 1) + [top] * dim, np.uint32)
    halves = ora.range_count_points(pts, np.array([lo_half, hi_half], np.uint32))
    assert int(halves.sum()) == len(pts)
