"""Structural invariants of a SPaC-tree exported from the GPU (test helper).

After updates the GPU structure depends on history (relaxed leaves, re-cut
leaves), so it is not compared with a canonical layout. Instead:
  I1  the sorted dump equals the oracle's set (checked by the caller);
  I2  pivots strictly increase and bracket every entry of their leaf:
      pivot_j <= e < pivot_{j+1} in (key, id) order;
  I3  every leaf holds between ceil(phi/2) and 2 phi entries (a single leaf
      may hold fewer);
  I4  leaf boxes are exactly tight; node boxes and counts are the union and
      sum of their children; the root counts every live point.
"""
import numpy as np

import oracle


def lex_less(ka, ia, kb, ib):
    return (ka < kb) | ((ka == kb) & (ia < ib))


def check(ix, phi, B, curve):
    st = ix.structure()
    L, h = st["n_leaves"], st["height"]
    ids, pts = ix.leaves()
    n = ids.size
    if L == 0:
        assert n == 0
        return st
    cnt = st["leaf_cnt"].astype(np.int64)
    assert cnt.sum() == n
    # I3
    if L > 1:
        assert cnt.min() >= (phi + 1) // 2, f"under-full leaf: {cnt.min()}"
    assert cnt.min() >= 1 and cnt.max() <= 2 * phi, (cnt.min(), cnt.max())
    starts = np.concatenate(([0], np.cumsum(cnt)[:-1]))
    owner = np.repeat(np.arange(L), cnt)
    # I4 leaves
    np.testing.assert_array_equal(st["leaf_lo"], np.minimum.reduceat(pts, starts, axis=0))
    np.testing.assert_array_equal(st["leaf_hi"], np.maximum.reduceat(pts, starts, axis=0))
    # I2
    pk, pi = st["piv_key"], st["piv_id"]
    assert np.all(lex_less(pk[:-1], pi[:-1], pk[1:], pi[1:])), "pivots not increasing"
    keys = oracle.encode(pts, ix.dim, curve)
    lo_ok = ~lex_less(keys, ids, pk[owner], pi[owner])
    assert lo_ok.all(), "entry below its leaf pivot"
    nxt = owner + 1
    has = nxt < L
    hi_ok = lex_less(keys[has], ids[has], pk[nxt[has]], pi[nxt[has]])
    assert hi_ok.all(), "entry not below the next pivot"
    # I4 nodes
    sizes = st["level_sizes"]
    offs = np.concatenate(([0], np.cumsum(sizes)))
    lo, hi, c = st["node_lo"], st["node_hi"], st["node_cnt"].astype(np.int64)
    np.testing.assert_array_equal(lo[offs[h]:offs[h + 1]], st["leaf_lo"])
    np.testing.assert_array_equal(c[offs[h]:offs[h + 1]], cnt)
    for lev in range(h):
        nchild = sizes[lev + 1]
        first = np.arange(0, nchild, B)
        sl = slice(offs[lev + 1], offs[lev + 2])
        np.testing.assert_array_equal(lo[offs[lev]:offs[lev + 1]], np.minimum.reduceat(lo[sl], first, axis=0))
        np.testing.assert_array_equal(hi[offs[lev]:offs[lev + 1]], np.maximum.reduceat(hi[sl], first, axis=0))
        np.testing.assert_array_equal(c[offs[lev]:offs[lev + 1]], np.add.reduceat(c[sl], first))
    assert c[0] == n
    return st
