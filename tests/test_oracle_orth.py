"""Pins of the P-Orth oracle (Sec. 3, Alg. 1) against definitions it must meet.

The oracle walks Alg. 1's steps (a lambda-level skeleton from region
midpoints, a sieve, recursion, merge-up). These tests check its result
against what an orth-tree is by definition, computed a different way: the
cells of a regular grid hierarchy taken straight from coordinate bits, one
level at a time, over all points (brute force). A wrong midpoint, a dropped
merge, a child order slip or a box error fails one of them.
"""
import numpy as np
import pytest

from oracle import orth

from synth import points


def cells(pts, dim, level):
    """Cell of every point at a level: low corner, from the coordinate bits."""
    W = orth.domain_bits(dim)
    sh = W - level
    return (pts >> sh) << sh


def brute_force_nodes(pts, dim, phi):
    """{(level, corner): (count, leaf)} of the canonical orth-tree: the root,
    and every non-empty cell whose parent cell holds more than phi points;
    a node is a leaf when it holds at most phi points or is a single grid
    point."""
    W = orth.domain_bits(dim)
    pts = np.asarray(pts, dtype=np.int64)
    out = {}
    if len(pts) == 0:
        return out
    out[(0, (0,) * dim)] = (len(pts), len(pts) <= phi)
    for level in range(1, W + 1):
        par = cells(pts, dim, level - 1)
        pu, pc = np.unique(par, axis=0, return_counts=True)
        big = {tuple(r) for r, c in zip(pu, pc) if c > phi}
        if not big:
            break
        cu, cc = np.unique(cells(pts, dim, level), axis=0, return_counts=True)
        pcell = cells(cu, dim, level - 1)
        for r, c, p in zip(cu, cc, pcell):
            if tuple(p) in big:
                out[(level, tuple(int(x) for x in r))] = (int(c), bool(c <= phi or level == W))
    return out


def tree_nodes(root):
    out = {}

    def walk(nd):
        out[(nd.level, tuple(int(x) for x in nd.corner))] = (nd.count, nd.leaf)
        for c in nd.children:
            walk(c)

    if root is not None:
        walk(root)
    return out


def inputs():
    yield "uniform2", 2, points("uniform", 3000, 2, bits=31, seed=1)
    yield "uniform3", 3, points("uniform", 3000, 3, bits=21, seed=2)
    yield "varden3", 3, points("varden", 3000, 3, bits=21, seed=3)
    yield "small-domain2", 2, points("uniform", 2000, 2, bits=6, seed=4)  # many equal points
    yield "sweepline2", 2, points("sweepline", 2000, 2, bits=31, seed=5)


@pytest.mark.parametrize("name,dim,pts", list(inputs()), ids=[x[0] for x in inputs()])
@pytest.mark.parametrize("phi", [2, 8, 32])
def test_tree_is_the_canonical_orth_tree(name, dim, pts, phi):
    root = orth.build(pts, dim, phi)
    assert tree_nodes(root) == brute_force_nodes(pts, dim, phi)


@pytest.mark.parametrize("name,dim,pts", list(inputs())[:3], ids=[x[0] for x in inputs()][:3])
def test_skeleton_height_does_not_change_the_tree(name, dim, pts):
    ref = orth.preorder(orth.build(pts, dim, 8, lam=1), dim)
    for lam in (2, 3, 5):
        got = orth.preorder(orth.build(pts, dim, 8, lam=lam), dim)
        for k in ("level", "corner", "leaf", "count", "lo", "hi", "end", "first"):
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"lam={lam} {k}")
        for a, b in zip(got["leaf_ids"], ref["leaf_ids"]):
            np.testing.assert_array_equal(np.sort(a), np.sort(b))


@pytest.mark.parametrize("name,dim,pts", list(inputs()), ids=[x[0] for x in inputs()])
def test_boxes_regions_and_leaves(name, dim, pts):
    phi = 8
    pts = np.asarray(pts, dtype=np.int64)
    W = orth.domain_bits(dim)
    pre = orth.preorder(orth.build(pts, dim, phi), dim)
    # every point in exactly one leaf; leaves cover the points in preorder
    all_ids = np.concatenate(pre["leaf_ids"])
    np.testing.assert_array_equal(np.sort(all_ids), np.arange(len(pts)))
    N = len(pre["level"])
    li = 0
    for v in range(N):
        side = 1 << (W - pre["level"][v])
        lo_r, hi_r = pre["corner"][v], pre["corner"][v] + side - 1
        # the subtree's points: the leaves between v and its end
        nl = int(pre["leaf"][v:pre["end"][v]].sum())
        ids = np.concatenate(pre["leaf_ids"][li:li + nl]) if pre["leaf"][v] or nl else np.zeros(0, np.int64)
        p = pts[ids]
        assert len(ids) == pre["count"][v]
        np.testing.assert_array_equal(pre["lo"][v], p.min(axis=0))
        np.testing.assert_array_equal(pre["hi"][v], p.max(axis=0))
        assert (p >= lo_r).all() and (p <= hi_r).all()  # inside the region
        if pre["leaf"][v]:
            assert pre["count"][v] <= phi or pre["level"][v] == W
            li += 1
        else:
            assert pre["count"][v] > phi
            # children: consecutive regions one level down, increasing index
            c, kids = v + 1, []
            while c < pre["end"][v]:
                kids.append(c)
                c = pre["end"][c]
            assert all(pre["level"][k] == pre["level"][v] + 1 for k in kids)
            half = side // 2
            idx = [sum(((pre["corner"][k][d] - pre["corner"][v][d]) // half) << d for d in range(dim)) for k in kids]
            assert idx == sorted(set(idx))
            assert pre["end"][kids[-1]] == pre["end"][v]


def test_empty_and_single_leaf():
    assert orth.build(np.zeros((0, 3), np.uint32), 3, 32) is None
    root = orth.build(points("uniform", 32, 3, bits=21, seed=9), 3, 32)
    assert root.leaf and root.level == 0 and root.count == 32


def test_equal_points_make_a_chain_to_one_grid_point():
    # phi + 5 copies of one point: every level splits off a single child down
    # to the grid point, which holds them all
    for dim in (2, 3):
        W = orth.domain_bits(dim)
        p = np.tile(np.array([[5, 9, 1][:dim]], dtype=np.uint32), (13, 1))
        pre = orth.preorder(orth.build(p, dim, 8), dim)
        assert len(pre["level"]) == W + 1
        np.testing.assert_array_equal(pre["level"], np.arange(W + 1))
        assert pre["leaf"].tolist() == [False] * W + [True]
        assert (pre["count"] == 13).all()
        assert (pre["end"] == W + 1).all()


def test_four_quadrants_by_hand():
    # 2D, phi = 2: three points in three quadrants of the domain -> the root
    # splits once; children in index order (x upper = bit 0, y upper = bit 1)
    h = 1 << 30
    p = np.array([[h + 1, 3], [2, h + 7], [h + 5, h + 5]], dtype=np.uint32)
    pre = orth.preorder(orth.build(p, 2, 2), 2)
    assert pre["leaf"].tolist() == [False, True, True, True]
    assert [tuple(c) for c in pre["corner"][1:]] == [(h, 0), (0, h), (h, h)]
    assert [a.tolist() for a in pre["leaf_ids"]] == [[0], [1], [2]]
    assert pre["end"].tolist() == [4, 2, 3, 4]
    assert pre["first"].tolist() == [-1, 0, 1, 2]


MUTANTS = [
    ("merge keeps subtrees of exactly phi points", "if nd.count <= phi:", "if nd.count < phi:"),
    ("a point on the midpoint goes low", "upper = p >= c + half", "upper = p > c + half"),
    ("children ordered with the axes swapped", "child |= upper[:, d].astype(np.int64) << d",
     "child |= upper[:, d].astype(np.int64) << (dim - 1 - d)"),
    ("box from the region, not the points", "nd.lo = p.min(axis=0)", "nd.lo = np.asarray(corner, dtype=np.int64)"),
    ("one-point cells split", "if len(ids) < phi or level == W:", "if len(ids) < phi or level == W + 1:"),
]


@pytest.mark.parametrize("what,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_a_planted_mistake(what, old, new):
    """Each plausible slip, planted in a copy of the oracle, fails a pin."""
    import types
    src = open(orth.__file__).read()
    assert old in src
    mod = types.ModuleType("orth_mutant")
    exec(compile(src.replace(old, new), "orth_mutant", "exec"), mod.__dict__)
    caught = False
    for name, dim, pts in inputs():
        for phi in (2, 8, 32):
            try:
                root = mod.build(pts, dim, phi)
                if tree_nodes(root) != brute_force_nodes(pts, dim, phi):
                    caught = True
                    break
                pre = mod.preorder(root, dim)
                p = np.asarray(pts, dtype=np.int64)
                for v in range(len(pre["level"])):
                    if pre["leaf"][v]:
                        j = int(pre["leaf"][:v].sum())
                        q = p[pre["leaf_ids"][j]]
                        if (pre["lo"][v] != q.min(axis=0)).any():
                            caught = True
                            break
            except Exception:
                caught = True
            if caught:
                break
        if caught:
            break
    assert caught, what


# ------------------------------------------------ batch updates (Alg. 2)
def check_canonical(root, rows, allp, dim, phi):
    """root is the orth-tree of the points allp[rows] by the definition (the
    brute-force cells), its leaves hold exactly those rows, and every node's
    box is the bounding box of its subtree's points."""
    p = allp[rows]
    assert tree_nodes(root) == brute_force_nodes(p, dim, phi)
    pre = orth.preorder(root, dim)
    got = np.sort(np.concatenate(pre["leaf_ids"])) if pre["leaf_ids"] else np.zeros(0, np.int64)
    np.testing.assert_array_equal(got, np.sort(np.asarray(rows, dtype=np.int64)))
    li = 0
    for v in range(len(pre["level"])):
        nl = int(pre["leaf"][v:pre["end"][v]].sum())
        ids = np.concatenate(pre["leaf_ids"][li:li + nl])
        np.testing.assert_array_equal(pre["lo"][v], allp[ids].min(axis=0))
        np.testing.assert_array_equal(pre["hi"][v], allp[ids].max(axis=0))
        assert pre["count"][v] == len(ids)
        if pre["leaf"][v]:
            li += 1


def update_script(dim, n, seed):
    """Seeded rows for a build, three insert batches (one of a single point)
    and three delete batches (one with repeats and rows never in the tree
    or already deleted)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    base, rest = perm[: n * 6 // 10], perm[n * 6 // 10:]
    ins = [rest[:1], rest[1:len(rest) // 2], rest[len(rest) // 2:]]
    live = np.sort(perm)
    d1 = rng.choice(live, n // 3, replace=False)
    left = np.setdiff1d(live, d1)
    d2 = np.concatenate([rng.choice(left, n // 5, replace=False), d1[:50], d1[:50], rng.choice(left, 20)])
    return base, ins, [d1, d2]


def run_updates(mod, name, dim, pts, phi):
    allp = np.asarray(pts, dtype=np.int64)
    base, ins, dels = update_script(dim, len(allp), seed=len(allp) + phi)
    root = mod.build(allp, dim, phi, ids=base)
    rows = np.asarray(base)
    yield root, rows
    for b in ins:
        root = mod.batch_insert(root, allp, b, dim, phi)
        rows = np.concatenate([rows, b])
        yield root, rows
    for d in dels:
        root = mod.batch_delete(root, allp, d, dim, phi)
        rows = np.setdiff1d(rows, d)
        yield root, rows
    root = mod.batch_delete(root, allp, rows, dim, phi)  # everything
    yield root, rows[:0]


@pytest.mark.parametrize("name,dim,pts", list(inputs()), ids=[x[0] for x in inputs()])
@pytest.mark.parametrize("phi", [2, 8, 32])
def test_alg2_updates_give_the_canonical_tree(name, dim, pts, phi):
    """Alg. 2's insertions (a leaf rebuilt by Alg. 1, skeletons sieving the
    batch) and deletions (removal at the leaves, ancestors of at most phi
    points flattened) reach the orth-tree of the new point set: the tree is
    canonical, which is what lets the GPU path cut the tree again from the
    merged order instead of updating it in place."""
    allp = np.asarray(pts, dtype=np.int64)
    for root, rows in run_updates(orth, name, dim, pts, phi):
        if len(rows) == 0:
            assert root is None
        else:
            check_canonical(root, rows, allp, dim, phi)


def test_alg2_skeleton_height_and_sharing():
    """Updates do not depend on the skeleton height, and leave their input
    tree unchanged."""
    dim, phi = 3, 8
    allp = np.asarray(points("varden", 3000, 3, bits=21, seed=3), dtype=np.int64)
    base, ins, dels = update_script(dim, len(allp), seed=77)
    t0 = orth.build(allp, dim, phi, ids=base)
    before = orth.preorder(t0, dim)
    ref = orth.preorder(orth.batch_delete(orth.batch_insert(t0, allp, ins[2], dim, phi, lam=1), allp, dels[0],
                                          dim, phi, lam=1), dim)
    for lam in (2, 4):
        got = orth.preorder(orth.batch_delete(orth.batch_insert(t0, allp, ins[2], dim, phi, lam=lam), allp, dels[0],
                                              dim, phi, lam=lam), dim)
        for k in ("level", "corner", "leaf", "count", "lo", "hi", "end", "first"):
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"lam={lam} {k}")
    after = orth.preorder(t0, dim)
    for k in ("level", "corner", "leaf", "count", "lo", "hi", "end", "first"):
        np.testing.assert_array_equal(after[k], before[k])


UPDATE_MUTANTS = [
    ("deletions never flatten", "if nd.count <= phi:  # flatten", "if nd.count < 0:  # flatten"),
    ("a leaf takes its share without Alg. 1",
     "return _build_region(pts, np.concatenate([node.ids, ids]), corner, level, dim, phi, lam)",
     "return _leaf(pts, np.concatenate([node.ids, ids]), level, corner)"),
    ("skeleton boxes not updated", "nd.lo = np.min([k.lo for k in kids], axis=0)", "nd.lo = kids[0].lo"),
    ("an emptied leaf kept", "return _leaf(pts, keep, level, corner) if len(keep) else None",
     "return _leaf(pts, keep if len(keep) else node.ids, level, corner)"),
    ("a point on the midpoint sieved low",
     "child |= (p[:, d] >= corner[d] + half).astype(np.int64) << d",
     "child |= (p[:, d] > corner[d] + half).astype(np.int64) << d"),
]


@pytest.mark.parametrize("what,old,new", UPDATE_MUTANTS, ids=[m[0] for m in UPDATE_MUTANTS])
def test_update_pins_catch_a_planted_mistake(what, old, new):
    """Each plausible slip in Alg. 2's oracle, planted in a copy, fails the
    update pins."""
    import types
    src = open(orth.__file__).read()
    assert old in src
    mod = types.ModuleType("orth_update_mutant")
    exec(compile(src.replace(old, new), "orth_update_mutant", "exec"), mod.__dict__)
    caught = False
    for name, dim, pts in inputs():
        allp = np.asarray(pts, dtype=np.int64)
        for phi in (2, 8):
            try:
                for root, rows in run_updates(mod, name, dim, pts, phi):
                    if len(rows) == 0:
                        assert root is None
                    else:
                        check_canonical(root, rows, allp, dim, phi)
            except AssertionError:
                caught = True
            except Exception:
                caught = True
            if caught:
                break
        if caught:
            break
    assert caught, what
