"""Pins of the paper-exact SPaC-tree oracle (oracle/spac.py): Alg. 3's
BuildSorted shape, Alg. 4's join-based batch insertion and the deletion that
mirrors it, App. C's leaf wrap and local-rebuild threshold.

What fixes them independently of the oracle's code:
  * Fig. 1's caption: 15 points with a leaf wrap of 3 give four leaves of 3
    points and 3 interior pivots;
  * BuildSorted's shape follows from n alone: leaf counts obey
    L(n) = 1 (n <= phi), L(floor(n/2)) + L(n - floor(n/2) - 1) otherwise, and
    the leaves are the sorted runs that recursion cuts;
  * the in-order sequence of any tree is the (key, id) sort of its point set,
    computed here by numpy's lexsort of the oracle's keys; the point set after
    updates is kept by a plain Python set;
  * every box equals the brute-force bounding box of its subtree's points;
  * weight balance (alpha = 0.2), the leaf wrap (leaves <= phi, interior
    nodes > phi) and BST order hold after every join and update.
Planted slips (in a monkeypatched copy of a function) must each fail a pin.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import spac


def runs(n, phi, a=0):
    """BuildSorted's leaves over sorted positions [a, a + n) and its
    pivots, written as the recursion's index arithmetic."""
    if n <= phi:
        return [("leaf", a, a + n)]
    m = n // 2
    return [("node", a + m)] + runs(m, phi, a) + runs(n - m - 1, phi, a + m + 1)


def leaf_count(n, phi):
    return 1 if n <= phi else leaf_count(n // 2, phi) + leaf_count(n - n // 2 - 1, phi)


def sorted_ids(pts, dim, curve):
    keys = oracle.encode(pts, dim, curve)
    ids = np.arange(len(pts), dtype=np.uint32)
    return ids[np.lexsort((ids, keys))]


def test_fig1_fifteen_points_wrap_three():
    # Fig. 1: 15 points, leaf wrap 3 -> 4 leaves of 3 points and 3 pivots
    pts = synth.uniform(15, 2, 10, seed=1)
    t = spac.SpacTree(2, oracle.HILBERT, phi=3).build(pts)
    pre = t.preorder()
    assert [k for k, *_ in pre] == [0, 0, 1, 1, 0, 1, 1]
    order = sorted_ids(pts, 2, oracle.HILBERT)
    assert pre[0][1] == order[7] and pre[1][1] == order[3] and pre[4][1] == order[11]
    leaves = [set(v) for k, v, *_ in pre if k == 1]
    assert leaves == [set(order[0:3]), set(order[4:7]), set(order[8:11]), set(order[12:15])]
    assert [s for k, _, s, *_ in pre] == [15, 7, 3, 3, 7, 3, 3]
    t.check()


@pytest.mark.parametrize("n,phi", [(0, 4), (1, 4), (4, 4), (5, 4), (40, 40), (41, 40), (100, 3), (1000, 40),
                                   (4097, 32), (777, 8)])
def test_build_sorted_shape(n, phi):
    pts = synth.uniform(n, 3, 21, seed=n + phi)
    t = spac.SpacTree(3, oracle.MORTON, phi=phi).build(pts)
    order = sorted_ids(pts, 3, oracle.MORTON)
    want = runs(n, phi)
    got = t.preorder()
    assert len(got) == len(want)
    for g, w in zip(got, want):
        if w[0] == "node":
            assert g[0] == 0 and g[1] == order[w[1]]
        else:
            assert g[0] == 1 and set(g[1]) == set(order[w[1]:w[2]])
    assert sum(1 for g in got if g[0] == 1) == leaf_count(n, phi)
    t.check()


def subtree_points(t):
    return spac.flatten(t)[2]


def check_boxes(t, dim):
    """Every box is the brute-force bounding box of its subtree's points."""
    def rec(x):
        p = subtree_points(x)
        lo, hi = spac.box(x, dim)
        if len(p):
            assert lo == tuple(int(v) for v in p.min(0)) and hi == tuple(int(v) for v in p.max(0))
        else:
            assert lo == (0xFFFFFFFF,) * dim and hi == (0,) * dim
        if isinstance(x, spac.Node):
            rec(x.left)
            rec(x.right)
    rec(t.root)


def test_boxes_cover_pivots():
    pts = synth.uniform(300, 2, 16, seed=3)
    t = spac.SpacTree(2, oracle.HILBERT, phi=4).build(pts)
    check_boxes(t, 2)


def in_order_matches(t):
    k, i, _ = spac.flatten(t.root)
    ids, pts = t.live()
    keys = oracle.encode(pts, t.dim, t.curve) if len(ids) else np.zeros(0, np.uint64)
    o = np.lexsort((ids, keys))
    np.testing.assert_array_equal(i, ids[o])
    np.testing.assert_array_equal(k, keys[o])


@pytest.mark.parametrize("na,nb", [(0, 0), (0, 50), (50, 0), (3, 200), (200, 3), (1000, 7), (64, 64), (500, 120)])
def test_join_keeps_order_and_balance(na, nb):
    # two trees over disjoint key ranges and a middle entry between them
    pts = synth.uniform(na + nb + 1, 2, 14, seed=na * 7 + nb)
    keys = oracle.encode(pts, 2, oracle.MORTON)
    ids = np.arange(len(pts), dtype=np.uint32)
    o = np.lexsort((ids, keys))
    k, i, p = keys[o], ids[o], pts[o]
    t = spac.SpacTree(2, oracle.MORTON, phi=6)
    a = t.build_sorted(k[:na], i[:na], p[:na])
    b = t.build_sorted(k[na + 1:], i[na + 1:], p[na + 1:])
    t.root = t.join(a, (int(k[na]), int(i[na]), p[na]), b)
    t.key_of = {int(x): int(y) for x, y in zip(ids, keys)}
    t.pt_of = {int(x): pts[int(x)] for x in ids}
    t.check()
    in_order_matches(t)
    check_boxes(t, 2)


@pytest.mark.parametrize("phi,curve,seed", [(3, 0, 1), (8, 1, 2), (40, 1, 3), (4, 0, 4)])
def test_updates_keep_invariants(phi, curve, seed):
    rng = np.random.default_rng(seed)
    t = spac.SpacTree(2, curve, phi=phi)
    n0 = int(rng.integers(0, 2000))
    t.build(synth.uniform(n0, 2, 12, seed))
    model = set(range(n0))
    for step in range(10):
        if rng.random() < 0.55:
            m = int(rng.choice([1, 3, 4 * phi, 5 * phi, 400, 2500]))
            new = t.batch_insert(synth.uniform(m, 2, 12, seed * 100 + step))
            model |= set(int(x) for x in new)
        else:
            live = np.array(sorted(model), np.uint32)
            ask = np.concatenate([rng.choice(live, int(rng.integers(0, len(live) + 1)), replace=False)
                                  if len(live) else np.zeros(0, np.uint32), [t.next_id + 5, 0, 0]])
            nd = t.batch_delete(ask)
            gone = {int(x) for x in ask} & model
            assert nd == len(gone)
            model -= gone
        t.check()
        assert set(int(x) for x in t.live()[0]) == model
        assert t.size() == len(model)
        in_order_matches(t)
    check_boxes(t, 2)


@pytest.mark.parametrize("dim,bits", [(2, 30), (3, 21)])
def test_full_width_keys_survive_updates(dim, bits):
    # keys above 2^53 (30-bit 2D and 21-bit 3D coordinates) stay exact
    # through flattening, Node()'s concatenation and deletes of pivots
    rng = np.random.default_rng(dim)
    t = spac.SpacTree(dim, oracle.HILBERT, phi=6).build(synth.uniform(300, dim, bits, 5))
    for step in range(8):
        if step % 2 == 0:
            t.batch_insert(synth.uniform(int(rng.integers(1, 200)), dim, bits, 50 + step))
        else:
            live = t.live()[0]
            t.batch_delete(rng.choice(live, len(live) // 2, replace=False))
        t.check()
        assert t.size() == len(t.live()[0])
        in_order_matches(t)


def test_expose_path_of_a_large_batch():
    # a leaf of 5 points and a batch of 40 at phi = 8: 45 >= 4 phi, so the
    # leaf is exposed and the batch inserted below it (App. C)
    t = spac.SpacTree(2, oracle.HILBERT, phi=8).build(synth.uniform(5, 2, 12, 1))
    assert isinstance(t.root, spac.Leaf)
    t.batch_insert(synth.uniform(40, 2, 12, 2))
    t.check()
    in_order_matches(t)
    assert isinstance(t.root, spac.Node) and t.size() == 45


def test_deleting_pivots_joins_both_sides():
    t = spac.SpacTree(2, oracle.MORTON, phi=4).build(synth.uniform(500, 2, 12, 9))
    piv = [v for k, v, *_ in t.preorder() if k == 0]
    t.batch_delete(np.array(piv[: len(piv) // 2], np.uint32))
    t.check()
    in_order_matches(t)
    assert t.size() == 500 - len(piv) // 2


# ------------------------------------------------------- planted slips fail
def _updates_pass(tree_cls_patch, monkeypatch):
    for name, fn in tree_cls_patch.items():
        monkeypatch.setattr(spac.SpacTree, name, fn)
    try:
        test_fig1_fifteen_points_wrap_three()
        for args in [(3, 0, 1), (8, 1, 2)]:
            test_updates_keep_invariants(*args)
        test_boxes_cover_pivots()
        test_join_keeps_order_and_balance(1000, 7)
        return True
    except (AssertionError, IndexError, ValueError, RecursionError):
        return False


def test_slip_split_position(monkeypatch):
    orig = spac.SpacTree.build_sorted

    def bad(self, keys, ids, pts):
        n = len(ids)
        if n <= self.phi:
            return spac.Leaf(keys, ids, pts, True)
        m = (n + 1) // 2  # slip: pivot one past the middle
        return spac.Node(bad(self, keys[:m], ids[:m], pts[:m]), int(keys[m]), int(ids[m]), pts[m],
                         bad(self, keys[m + 1:], ids[m + 1:], pts[m + 1:]))
    assert not _updates_pass({"build_sorted": bad}, monkeypatch)
    monkeypatch.setattr(spac.SpacTree, "build_sorted", orig)


def test_slip_no_rotation(monkeypatch):
    def bad(self, tl, kp, tr):  # slip: join down the spine without rebalancing
        if spac.like(spac.weight(tl), spac.weight(tr), self.alpha):
            return self.node(tl, *kp, tr)
        l, k2, c = self.expose(tl)
        return self.node(l, *k2, bad(self, c, kp, tr))
    assert not _updates_pass({"join_right": bad}, monkeypatch)


def test_slip_node_never_wraps(monkeypatch):
    def bad(self, left, key, id_, pt, right):  # slip: small subtrees stay interior nodes
        return spac.Node(left, key, id_, pt, right)
    assert not _updates_pass({"node": bad}, monkeypatch)


def test_slip_box_without_pivot(monkeypatch):
    orig = spac.box

    def bad(t, dim):
        if isinstance(t, spac.Leaf):
            return orig(t, dim)
        llo, lhi = bad(t.left, dim)
        rlo, rhi = bad(t.right, dim)
        return tuple(min(a, b) for a, b in zip(llo, rlo)), tuple(max(a, b) for a, b in zip(lhi, rhi))
    monkeypatch.setattr(spac, "box", bad)
    with pytest.raises(AssertionError):
        test_boxes_cover_pivots()
