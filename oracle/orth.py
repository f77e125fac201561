"""P-Orth tree oracle (Sec. 3, Alg. 1), plain numpy and Python recursion.

TEST INFRASTRUCTURE ONLY: the test suite is the only user. The product path
never imports this module.

Alg. 1 (BuildOrth) on a point set P and its region H:
  * |P| < phi: a leaf holding P;
  * otherwise a skeleton of lambda levels below H (lambda = 3 in 2D, 2 in 3D,
    App. C), the sub-region of each of its 2^(lambda D) external nodes, a
    sieve of P into those buckets (a stable counting sort by bucket), a
    recursive build per non-empty bucket, then the boxes of the skeleton's
    internal nodes and the merge of every subtree of at most phi points into
    one leaf.

Readings where the paper is silent (listed with the others in the design
notes):
  * the root region is the coordinate domain [0, 2^W)^D (W = 31 in 2D, 21 in
    3D), so every region is a cell of a regular grid hierarchy;
  * a region is split at its midpoint on every axis, a point going to the
    upper half of axis d when its coordinate is at least the midpoint;
  * the children of a node are ordered by sub-region index
    sum_d [upper half on axis d] << d, empty sub-regions have no node;
  * a region of side 1 cannot be split: it is a leaf whatever its size;
  * a node's box is the bounding box of its points (App. C stores its two
    corners).
"""
from __future__ import annotations

import numpy as np


def domain_bits(dim: int) -> int:
    return 31 if dim == 2 else 21


class Node:
    __slots__ = ("level", "corner", "leaf", "ids", "children", "lo", "hi", "count")

    def __init__(self, level, corner):
        self.level = level
        self.corner = corner  # low corner of the region, tuple of ints
        self.leaf = False
        self.ids = None        # leaf: point ids
        self.children = []     # interior: non-empty sub-regions, in index order
        self.lo = self.hi = None
        self.count = 0


def _leaf(pts, ids, level, corner):
    nd = Node(level, corner)
    nd.leaf = True
    nd.ids = np.asarray(ids, dtype=np.int64)
    nd.count = len(nd.ids)
    p = pts[nd.ids]
    nd.lo = p.min(axis=0)
    nd.hi = p.max(axis=0)
    return nd


def _all_ids(nd):
    if nd.leaf:
        return nd.ids
    return np.concatenate([_all_ids(c) for c in nd.children])


def build(pts, dim: int, phi: int, lam: int | None = None, ids=None):
    """The P-Orth tree of `pts` (ids = row numbers), or of the rows `ids`
    alone when given; None when empty."""
    pts = np.asarray(pts, dtype=np.int64).reshape(-1, dim)
    ids = np.arange(len(pts), dtype=np.int64) if ids is None else np.asarray(ids, dtype=np.int64)
    if len(ids) == 0:
        return None
    return _build_region(pts, ids, tuple([0] * dim), 0, dim, phi, lam)


def _build_region(pts, ids, corner, level, dim: int, phi: int, lam: int | None = None):
    """Alg. 1 on the points `ids` (rows of pts) of the region with low corner
    `corner` at `level`; None when there are none."""
    W = domain_bits(dim)
    lam = lam if lam is not None else (3 if dim == 2 else 2)
    if len(ids) == 0:
        return None

    def build_orth(ids, corner, level):
        if len(ids) < phi or level == W:
            return _leaf(pts, ids, level, corner)
        h = min(lam, W - level)  # skeleton height (a side-1 region stops it)
        # skeleton walk: the bucket of each point, from the midpoints
        p = pts[ids]
        c = np.tile(np.asarray(corner, dtype=np.int64), (len(ids), 1))
        bucket = np.zeros(len(ids), dtype=np.int64)
        for j in range(h):
            half = 1 << (W - level - j - 1)
            upper = p >= c + half
            child = np.zeros(len(ids), dtype=np.int64)
            for d in range(dim):
                child |= upper[:, d].astype(np.int64) << d
            bucket = (bucket << dim) | child
            c = c + upper * half
        # sieve: points of a bucket made consecutive, order kept
        order = np.argsort(bucket, kind="stable")
        ids_s, b_s = ids[order], bucket[order]
        nb = 1 << (dim * h)
        starts = np.searchsorted(b_s, np.arange(nb + 1))
        # recursive build of every non-empty bucket
        sub = {}
        for b in range(nb):
            if starts[b] == starts[b + 1]:
                continue
            sc = list(corner)
            path = b
            for j in range(h):  # the bucket index is the path, top level first
                ch = (path >> (dim * (h - 1 - j))) & ((1 << dim) - 1)
                half = 1 << (W - level - j - 1)
                for d in range(dim):
                    if (ch >> d) & 1:
                        sc[d] += half
            sub[b] = build_orth(ids_s[starts[b]:starts[b + 1]], tuple(sc), level + h)

        # skeleton's internal nodes (post-order): boxes, then merge-up
        def assemble(prefix, depth, cor):
            if depth == h:
                return sub.get(prefix)
            kids = []
            half = 1 << (W - level - depth - 1)
            for ch in range(1 << dim):
                cc = tuple(cor[d] + (half if (ch >> d) & 1 else 0) for d in range(dim))
                k = assemble((prefix << dim) | ch, depth + 1, cc)
                if k is not None:
                    kids.append(k)
            if not kids:
                return None
            nd = Node(level + depth, tuple(cor))
            nd.children = kids
            nd.count = sum(k.count for k in kids)
            nd.lo = np.min([k.lo for k in kids], axis=0)
            nd.hi = np.max([k.hi for k in kids], axis=0)
            if nd.count <= phi:  # merge a small subtree into one leaf
                return _leaf(pts, _all_ids(nd), nd.level, nd.corner)
            return nd

        return assemble(0, 0, tuple(corner))

    return build_orth(np.asarray(ids, dtype=np.int64), tuple(corner), level)


def _interior(level, corner, kids):
    nd = Node(level, corner)
    nd.children = kids
    nd.count = sum(k.count for k in kids)
    nd.lo = np.min([k.lo for k in kids], axis=0)
    nd.hi = np.max([k.hi for k in kids], axis=0)
    return nd


def _sieve_children(pts, ids, node, corner, level, dim):
    """Sec. 3.2's sieve one level down: for each sub-region of the region
    (index sum_d [upper half on axis d] << d), its low corner, the existing
    child there (None when empty) and the slice of `ids` that falls in it,
    order kept."""
    W = domain_bits(dim)
    half = 1 << (W - level - 1)
    p = pts[ids]
    child = np.zeros(len(ids), dtype=np.int64)
    for d in range(dim):
        child |= (p[:, d] >= corner[d] + half).astype(np.int64) << d
    existing = {}
    if node is not None:
        for c in node.children:
            idx = sum(((c.corner[d] - corner[d]) // half) << d for d in range(dim))
            existing[idx] = c
    for ch in range(1 << dim):
        sc = tuple(corner[d] + (half if (ch >> d) & 1 else 0) for d in range(dim))
        yield sc, existing.get(ch), ids[child == ch]


def batch_insert(root, pts, new_ids, dim: int, phi: int, lam: int | None = None):
    """Alg. 2 (batch insertion): the points `new_ids` (rows of pts, not in the
    tree) added to the tree `root` of other rows of pts. An empty batch leaves
    a subtree as it is; a leaf takes Alg. 1 again on its points and the
    batch's; an interior node's skeleton (lambda levels of its subtree) sieves
    the batch to its external nodes, each of which takes its share the same
    way (an empty sub-region gets Alg. 1 on its share); the boxes of the
    skeleton's nodes are then updated. `root` is not modified (the subtrees
    the batch does not reach are shared with the tree returned)."""
    pts = np.asarray(pts, dtype=np.int64).reshape(-1, dim)
    W = domain_bits(dim)
    lam = lam if lam is not None else (3 if dim == 2 else 2)
    new_ids = np.asarray(new_ids, dtype=np.int64)

    def insert(node, ids, corner, level):
        if len(ids) == 0:
            return node
        if node is None:
            return _build_region(pts, ids, corner, level, dim, phi, lam)
        if node.leaf:
            return _build_region(pts, np.concatenate([node.ids, ids]), corner, level, dim, phi, lam)
        return skeleton(node, ids, corner, level, min(lam, W - level))

    def skeleton(node, ids, corner, level, h):
        # the skeleton's nodes down to h levels below; its external nodes
        # (leaves, empty sub-regions, nodes h levels down) take their shares
        if len(ids) == 0:  # nothing below changes
            return node
        if h == 0 or node is None or node.leaf:
            return insert(node, ids, corner, level)
        kids = []
        for sc, c, share in _sieve_children(pts, ids, node, corner, level, dim):
            t = skeleton(c, share, sc, level + 1, h - 1)
            if t is not None:
                kids.append(t)
        return _interior(level, corner, kids)

    if root is None:
        return build(pts, dim, phi, lam, ids=new_ids)
    return insert(root, new_ids, tuple([0] * dim), 0)


def batch_delete(root, pts, del_ids, dim: int, phi: int, lam: int | None = None):
    """Alg. 2's deletion (symmetric to insertion, Sec. 3.2): the rows
    `del_ids` (coordinates from pts) are sieved down the skeletons to the
    leaves that hold them and removed there (ids the tree does not hold are
    ignored); a node left without points disappears, and every affected
    ancestor whose subtree holds at most phi points is flattened into one
    leaf. `root` is not modified (the subtrees the batch does not reach are
    shared with the tree returned)."""
    pts = np.asarray(pts, dtype=np.int64).reshape(-1, dim)
    W = domain_bits(dim)
    lam = lam if lam is not None else (3 if dim == 2 else 2)
    del_ids = np.unique(np.asarray(del_ids, dtype=np.int64))

    def delete(node, ids, corner, level):
        if node is None or len(ids) == 0:
            return node
        if node.leaf:
            keep = node.ids[~np.isin(node.ids, ids)]
            if len(keep) == len(node.ids):
                return node
            return _leaf(pts, keep, level, corner) if len(keep) else None
        return skeleton(node, ids, corner, level, min(lam, W - level))

    def skeleton(node, ids, corner, level, h):
        if len(ids) == 0:  # nothing below changes
            return node
        if h == 0 or node is None or node.leaf:
            return delete(node, ids, corner, level)
        kids = []
        for sc, c, share in _sieve_children(pts, ids, node, corner, level, dim):
            t = skeleton(c, share, sc, level + 1, h - 1) if c is not None else None
            if t is not None:
                kids.append(t)
        if not kids:
            return None
        nd = _interior(level, corner, kids)
        if nd.count <= phi:  # flatten a subtree the deletions brought down to phi points
            return _leaf(pts, _all_ids(nd), level, corner)
        return nd

    return skeleton(root, del_ids, tuple([0] * dim), 0, min(lam, W)) if root is not None else None


def preorder(root, dim: int, ids=None) -> dict:
    """Depth-first preorder arrays of a tree (children in index order):
    level, corner, leaf flag, count, lo, hi, end (index one past the subtree),
    first (first point of a leaf in leaf order) and the leaves' id arrays
    (row numbers of the built points, or ids[row] when ids is given)."""
    out = dict(level=[], corner=[], leaf=[], count=[], lo=[], hi=[], end=[], first=[], leaf_ids=[])
    if root is None:
        for k in ("level", "count", "end", "first"):
            out[k] = np.zeros(0, dtype=np.int64)
        out["leaf"] = np.zeros(0, dtype=bool)
        for k in ("lo", "hi", "corner"):
            out[k] = np.zeros((0, dim), dtype=np.int64)
        return out
    pos = [0]

    def walk(nd):
        v = len(out["level"])
        out["level"].append(nd.level)
        out["corner"].append(nd.corner)
        out["leaf"].append(nd.leaf)
        out["count"].append(nd.count)
        out["lo"].append(nd.lo)
        out["hi"].append(nd.hi)
        out["end"].append(-1)
        out["first"].append(pos[0] if nd.leaf else -1)
        if nd.leaf:
            out["leaf_ids"].append(nd.ids if ids is None else np.asarray(ids, dtype=np.int64)[nd.ids])
            pos[0] += nd.count
        else:
            for c in nd.children:
                walk(c)
        out["end"][v] = len(out["level"])

    walk(root)
    for k in ("level", "count", "end", "first"):
        out[k] = np.asarray(out[k], dtype=np.int64)
    out["leaf"] = np.asarray(out["leaf"], dtype=bool)
    for k in ("lo", "hi", "corner"):
        out[k] = np.asarray(out[k], dtype=np.int64).reshape(-1, dim)
    return out
