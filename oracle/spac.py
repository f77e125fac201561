"""Oracle of the paper-exact SPaC-tree shape and its join-based batch updates
(Sec. 4: Alg. 3's BuildSorted, Alg. 4's BatchInsert with Join, RightJoin,
LeftJoin, Expose and Node; App. C's leaf wrap and local-rebuild threshold).
Plain Python recursion over numpy arrays, for small inputs.

TEST INFRASTRUCTURE ONLY: the test suite is the only user. The product path
never imports this module.

The tree is a binary search tree on (curve key, id) whose subtrees of at
most phi points are wrapped into leaves (arrays of points, possibly out of
key order after appends). An interior node holds one point, its pivot.
Readings where the paper is silent or loose (listed with the others in the
design notes):
  * BuildSorted on n > phi sorted entries puts entry m = floor(n / 2) in the
    node, entries [0, m) left and [m + 1, n) right;
  * weight = size + 1; a pair of subtrees is balanced when the lighter one
    weighs at least alpha of both together (the usual weight-balance rule;
    alpha = 0.2 as App. C sets it);
  * Expose of a leaf sorts it if needed and splits it like BuildSorted's
    first step: leaf [0, m), pivot m, leaf [m + 1, n);
  * Node(L, k, R) over n points: an interior node if n > 2 phi; two sorted
    leaves split like BuildSorted's first step if phi < n <= 2 phi; one leaf
    otherwise (sorted if both sides were);
  * a leaf that would overflow takes a local rebuild (BuildSorted of its
    points and the batch's) when both together hold fewer than 4 phi points,
    else it is exposed and the batch inserted into the exposed subtree;
  * an interior node's box covers its children's boxes and its own pivot;
  * deletion follows insertion's recursion; a deleted pivot is replaced by
    joining its two sides without a middle key (the last point of the left
    side moves up).
"""
from __future__ import annotations

import numpy as np

from . import encode


class Leaf:
    __slots__ = ("keys", "ids", "pts", "sorted")

    def __init__(self, keys, ids, pts, is_sorted=True):
        self.keys, self.ids, self.pts, self.sorted = keys, ids, pts, is_sorted


class Node:
    __slots__ = ("left", "right", "key", "id", "pt", "size")

    def __init__(self, left, key, id_, pt, right):
        self.left, self.right, self.key, self.id, self.pt = left, right, key, id_, pt
        self.size = size(left) + 1 + size(right)


def size(t) -> int:
    return len(t.ids) if isinstance(t, Leaf) else t.size


def weight(t) -> int:
    return size(t) + 1


def like(wa: int, wb: int, alpha: float) -> bool:
    """Two subtree weights are balanced."""
    return alpha * (wa + wb) <= min(wa, wb)


def _order(keys, ids):
    return np.lexsort((ids, keys))


def _empty(dim):
    return Leaf(np.zeros(0, np.uint64), np.zeros(0, np.uint32), np.zeros((0, dim), np.uint32))


def _sorted_leaf(t: Leaf) -> Leaf:
    if t.sorted:
        return t
    o = _order(t.keys, t.ids)
    return Leaf(t.keys[o], t.ids[o], t.pts[o], True)


def flatten(t):
    """All entries of a subtree in (key, id) order."""
    if isinstance(t, Leaf):
        s = _sorted_leaf(t)
        return s.keys, s.ids, s.pts
    lk, li, lp = flatten(t.left)
    rk, ri, rp = flatten(t.right)
    # the keys stay 64-bit integers (a Python int beside a uint64 array would
    # promote the concatenation to floating point and round keys above 2^53)
    return (np.concatenate([lk, np.array([t.key], np.uint64), rk]), np.concatenate([li, [t.id], ri]).astype(np.uint32),
            np.concatenate([lp, t.pt[None, :], rp]).astype(np.uint32))


class SpacTree:
    """The tree with its parameters (leaf wrap phi, balance alpha, 4 phi
    local-rebuild threshold) and the id table deletes need."""

    def __init__(self, dim: int, curve: int, phi: int = 40, alpha: float = 0.2):
        self.dim, self.curve, self.phi, self.alpha = dim, curve, phi, alpha
        self.root = _empty(dim)
        self.key_of = {}
        self.pt_of = {}
        self.next_id = 0

    # ---------------------------------------------------------------- build
    def build_sorted(self, keys, ids, pts):
        """Alg. 3's BuildSorted on entries already in (key, id) order."""
        n = len(ids)
        if n <= self.phi:
            return Leaf(keys, ids, pts, True)
        m = n // 2
        left = self.build_sorted(keys[:m], ids[:m], pts[:m])
        right = self.build_sorted(keys[m + 1:], ids[m + 1:], pts[m + 1:])
        return Node(left, int(keys[m]), int(ids[m]), pts[m], right)

    def build(self, pts):
        pts = np.ascontiguousarray(pts, np.uint32).reshape(-1, self.dim)
        n = len(pts)
        keys = encode(pts, self.dim, self.curve) if n else np.zeros(0, np.uint64)
        ids = np.arange(n, dtype=np.uint32)
        o = _order(keys, ids)
        self.root = self.build_sorted(keys[o], ids[o], pts[o])
        self.key_of = {int(i): int(k) for i, k in zip(ids, keys)}
        self.pt_of = {int(i): pts[int(i)] for i in ids}
        self.next_id = n
        return self

    # ------------------------------------------------- Alg. 4's join machinery
    def node(self, left, key, id_, pt, right):
        """Node(): a node that keeps the leaf wrap."""
        n = size(left) + 1 + size(right)
        if n > 2 * self.phi:
            return Node(left, key, id_, pt, right)
        both_leaves_sorted = (isinstance(left, Leaf) and left.sorted and isinstance(right, Leaf) and right.sorted)
        if n > self.phi:  # two leaves of about n / 2
            k, i, p = flatten(Node(left, key, id_, pt, right))
            m = n // 2
            return Node(Leaf(k[:m], i[:m], p[:m]), int(k[m]), int(i[m]), p[m], Leaf(k[m + 1:], i[m + 1:], p[m + 1:]))
        if isinstance(left, Leaf) and isinstance(right, Leaf):  # left < key < right: concatenation in place
            return Leaf(np.concatenate([left.keys, np.array([key], np.uint64), right.keys]),
                        np.concatenate([left.ids, [id_], right.ids]).astype(np.uint32),
                        np.concatenate([left.pts, pt[None, :], right.pts]).astype(np.uint32), both_leaves_sorted)
        k, i, p = flatten(Node(left, key, id_, pt, right))
        return Leaf(k, i, p, True)

    def expose(self, t):
        """(left, pivot, right) of a node; a leaf is sorted if needed and
        split like BuildSorted's first step. The leaf must not be empty."""
        if isinstance(t, Node):
            return t.left, (t.key, t.id, t.pt), t.right
        s = _sorted_leaf(t)
        m = len(s.ids) // 2
        return (Leaf(s.keys[:m], s.ids[:m], s.pts[:m]), (int(s.keys[m]), int(s.ids[m]), s.pts[m]),
                Leaf(s.keys[m + 1:], s.ids[m + 1:], s.pts[m + 1:]))

    def join(self, left, kp, right):
        a = self.alpha
        wl, wr = weight(left), weight(right)
        if not like(wl, wr, a):
            if wl > wr:
                return self.join_right(left, kp, right)
            return self.join_left(left, kp, right)
        return self.node(left, *kp, right)

    def join_right(self, tl, kp, tr):
        """tl heavier: walk down tl's right spine until a subtree balances
        with tr, join there, rebalance on the way back by rotations."""
        a = self.alpha
        if like(weight(tl), weight(tr), a):
            return self.node(tl, *kp, tr)
        l, k2, c = self.expose(tl)
        t2 = self.join_right(c, kp, tr)
        if like(weight(l), weight(t2), a):
            return self.node(l, *k2, t2)
        l1, k3, r1 = self.expose(t2)
        if (like(weight(l), weight(l1), a) and like(weight(l) + weight(l1), weight(r1), a)) or size(l1) == 0:
            return self.node(self.node(l, *k2, l1), *k3, r1)  # rotate left
        a1, k4, b1 = self.expose(l1)  # rotate t2 right, then left
        return self.node(self.node(l, *k2, a1), *k4, self.node(b1, *k3, r1))

    def join_left(self, tl, kp, tr):
        """The mirror of join_right (tr heavier)."""
        a = self.alpha
        if like(weight(tl), weight(tr), a):
            return self.node(tl, *kp, tr)
        c, k2, r = self.expose(tr)
        t2 = self.join_left(tl, kp, c)
        if like(weight(t2), weight(r), a):
            return self.node(t2, *k2, r)
        l1, k3, r1 = self.expose(t2)
        if (like(weight(r1), weight(r), a) and like(weight(r1) + weight(r), weight(l1), a)) or size(r1) == 0:
            return self.node(l1, *k3, self.node(r1, *k2, r))  # rotate right
        a1, k4, b1 = self.expose(r1)  # rotate t2 left, then right
        return self.node(self.node(l1, *k3, a1), *k4, self.node(b1, *k2, r))

    def split_last(self, t):
        """(t without its largest entry, that entry)."""
        if isinstance(t, Leaf):
            s = _sorted_leaf(t)
            return Leaf(s.keys[:-1], s.ids[:-1], s.pts[:-1]), (int(s.keys[-1]), int(s.ids[-1]), s.pts[-1])
        r2, kp = self.split_last(t.right)
        return self.join(t.left, (t.key, t.id, t.pt), r2), kp

    def join2(self, left, right):
        if size(left) == 0:
            return right
        l2, kp = self.split_last(left)
        return self.join(l2, kp, right)

    # -------------------------------------------------------------- updates
    def _insert(self, t, keys, ids, pts):
        n = len(ids)
        if n == 0:
            return t
        if isinstance(t, Leaf):
            m = len(t.ids)
            if m + n <= self.phi:  # append, order relaxed
                return Leaf(np.concatenate([t.keys, keys]).astype(np.uint64),
                            np.concatenate([t.ids, ids]).astype(np.uint32),
                            np.concatenate([t.pts, pts]).astype(np.uint32), m == 0)
            if m + n < 4 * self.phi or m == 0:  # local rebuild (nothing to expose in an empty leaf)
                k = np.concatenate([t.keys, keys]).astype(np.uint64)
                i = np.concatenate([t.ids, ids]).astype(np.uint32)
                p = np.concatenate([t.pts, pts]).astype(np.uint32)
                o = _order(k, i)
                return self.build_sorted(k[o], i[o], p[o])
            l, kp, r = self.expose(t)
            t = Node(l, kp[0], kp[1], kp[2], r)
        # entries below the pivot go left (ids are new: no entry equals it)
        tcut = int(np.searchsorted(_lex_rank(keys, ids, t.key, t.id), True))
        left = self._insert(t.left, keys[:tcut], ids[:tcut], pts[:tcut])
        right = self._insert(t.right, keys[tcut:], ids[tcut:], pts[tcut:])
        return self.join(left, (t.key, t.id, t.pt), right)

    def batch_insert(self, pts):
        """Alg. 4: sort the batch by (key, id), then insert it; returns ids."""
        pts = np.ascontiguousarray(pts, np.uint32).reshape(-1, self.dim)
        m = len(pts)
        ids = np.arange(self.next_id, self.next_id + m, dtype=np.uint32)
        keys = encode(pts, self.dim, self.curve) if m else np.zeros(0, np.uint64)
        for i, k, p in zip(ids, keys, pts):
            self.key_of[int(i)] = int(k)
            self.pt_of[int(i)] = p
        self.next_id += m
        o = _order(keys, ids)
        self.root = self._insert(self.root, keys[o], ids[o], pts[o])
        return ids

    def _delete(self, t, keys, ids):
        if len(ids) == 0:
            return t
        if isinstance(t, Leaf):
            keep = ~np.isin(t.ids, ids)
            return Leaf(t.keys[keep], t.ids[keep], t.pts[keep], t.sorted)
        rank = _lex_rank(keys, ids, t.key, t.id)  # True where the entry is not below the pivot
        tcut = int(np.searchsorted(rank, True))
        hit = tcut < len(ids) and int(keys[tcut]) == t.key and int(ids[tcut]) == t.id
        left = self._delete(t.left, keys[:tcut], ids[:tcut])
        right = self._delete(t.right, keys[tcut + hit:], ids[tcut + hit:])
        if hit:
            return self.join2(left, right)
        return self.join(left, (t.key, t.id, t.pt), right)

    def batch_delete(self, ids) -> int:
        """Deletes the live ids among `ids` (others ignored); returns how many."""
        live = sorted({int(i) for i in np.asarray(ids).ravel() if int(i) in self.key_of})
        if not live:
            return 0
        keys = np.array([self.key_of[i] for i in live], np.uint64)
        idv = np.array(live, np.uint32)
        o = _order(keys, idv)
        self.root = self._delete(self.root, keys[o], idv[o])
        for i in live:
            del self.key_of[i]
            del self.pt_of[i]
        return len(live)

    # ------------------------------------------------------------ inspection
    def size(self) -> int:
        return size(self.root)

    def live(self):
        """Live ids and their points, ids ascending."""
        ids = np.array(sorted(self.key_of), np.uint32)
        pts = np.array([self.pt_of[int(i)] for i in ids], np.uint32).reshape(-1, self.dim)
        return ids, pts

    def preorder(self):
        """The structure in preorder: (kind, pivot id or sorted leaf ids,
        size, box lo, box hi) per node; kind 0 = interior, 1 = leaf."""
        out = []

        def rec(t):
            lo, hi = box(t, self.dim)
            if isinstance(t, Leaf):
                out.append((1, tuple(sorted(int(i) for i in t.ids)), len(t.ids), lo, hi))
                return
            out.append((0, t.id, t.size, lo, hi))
            rec(t.left)
            rec(t.right)

        rec(self.root)
        return out

    def check(self):
        """The invariants: BST order on (key, id) with leaves as blocks, leaf
        wrap (leaves at most phi points, interior nodes more than phi),
        weight balance at every interior node; raises AssertionError."""
        phi, a = self.phi, self.alpha

        def rec(t):
            if isinstance(t, Leaf):
                assert len(t.ids) <= phi, f"leaf of {len(t.ids)} > phi"
                if t.sorted and len(t.ids) > 1:
                    o = _order(t.keys, t.ids)
                    assert np.array_equal(o, np.arange(len(o))), "leaf marked sorted is not"
                return
            assert t.size > phi, f"interior node of {t.size} <= phi"
            assert t.size == size(t.left) + 1 + size(t.right)
            assert like(weight(t.left), weight(t.right), a), (size(t.left), size(t.right))
            rec(t.left)
            rec(t.right)

        rec(self.root)
        k, i, _ = flatten(self.root)
        if len(k) > 1:
            ok = (k[:-1] < k[1:]) | ((k[:-1] == k[1:]) & (i[:-1] < i[1:]))
            assert ok.all(), "in-order is not increasing in (key, id)"


def _lex_rank(keys, ids, key, id_):
    """Boolean per entry (sorted by (key, id)): entry >= (key, id_)."""
    keys = np.asarray(keys, np.uint64)
    return (keys > np.uint64(key)) | ((keys == np.uint64(key)) & (np.asarray(ids, np.uint32) >= np.uint32(id_)))


def box(t, dim: int):
    """Bounding box of a subtree (its leaves' points and its pivots); an
    empty leaf has lo = 0xFFFFFFFF, hi = 0 on every axis."""
    if isinstance(t, Leaf):
        if len(t.ids) == 0:
            return (0xFFFFFFFF,) * dim, (0,) * dim
        return tuple(int(x) for x in t.pts.min(0)), tuple(int(x) for x in t.pts.max(0))
    llo, lhi = box(t.left, dim)
    rlo, rhi = box(t.right, dim)
    lo = tuple(min(a, b, int(c)) for a, b, c in zip(llo, rlo, t.pt))
    hi = tuple(max(a, b, int(c)) for a, b, c in zip(lhi, rhi, t.pt))
    return lo, hi
