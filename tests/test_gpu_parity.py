"""GPU parity: every step of the HIP path against the CPU oracle, bit-exact.

All inputs are seeded synthetic arrays from `synth`; every expected value
comes from the oracle. Sizes span several 4096-pair sort tiles with a ragged
tail; the full-size configurations are covered in test_gpu_fullsize.py.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CURVES = [(2, 0), (2, 1), (3, 0), (3, 1)]


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


def make_pair(psi, dim, curve, pts, phi=32, B=8):
    ix = psi.Index(dim, curve, phi, B)
    ix.build(pts)
    ref = oracle.RefIndex(dim, curve, phi, B)
    ref.build(pts)
    return ix, ref


# ------------------------------------------------------------------ encode
@pytest.mark.parametrize("dim,curve", CURVES)
def test_encode_parity(psi, dim, curve):
    say(f"encode dim={dim} curve={curve}")
    lim = 31 if dim == 2 else 21
    pts = synth.uniform(1_000_003, dim, lim, seed=100 + dim)
    corners = np.array(np.meshgrid(*([[0, (1 << lim) - 1]] * dim), indexing="ij")).reshape(dim, -1).T
    pts = np.concatenate([pts, corners.astype(np.uint32)])
    got = psi.to_u64(psi.encode(pts, dim, curve))
    np.testing.assert_array_equal(got, oracle.encode(pts, dim, curve))


@pytest.mark.parametrize("dim", [2, 3])
def test_encode_rejects_out_of_range(psi, dim):
    say(f"encode range dim={dim}")
    bad = np.zeros((5, dim), np.uint32)
    bad[3, dim - 1] = 1 << (31 if dim == 2 else 21)
    with pytest.raises(psi.PsiError) as e:
        psi.encode(bad, dim, 1)
    assert e.value.code == 2


# -------------------------------------------------------------------- sort
@pytest.mark.parametrize("n", [1, 4095, 4096, 4097, 10_240, 10_241, 300_007])  # 10240: the one-workgroup sort's limit
def test_sort_pairs_parity(psi, n):
    say(f"sort n={n}")
    r = synth.draws(synth.stream_key(n, 9), 0, 2 * n)
    keys = r[:n] >> np.uint64(40)            # many equal keys
    keys[::7] = r[n:][::7]                    # and some full 64-bit keys
    ids = np.argsort(r[n:], kind="stable").astype(np.uint32)  # ids in random order
    k, i = psi.sort_pairs(keys, ids)
    ek, ei = oracle.sort_pairs(keys, ids)
    np.testing.assert_array_equal(psi.to_u64(k), ek)
    np.testing.assert_array_equal(psi.to_u32(i), ei)


# ------------------------------------------------------------------- build
@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 1000, 100_003])
@pytest.mark.parametrize("dim,curve", CURVES)
def test_build_structure_parity(psi, dim, curve, n):
    say(f"build dim={dim} curve={curve} n={n}")
    pts = synth.uniform(n, dim, bits_of(dim), seed=n + 3)
    ix, ref = make_pair(psi, dim, curve, pts)
    g, e = ix.structure(), ref.structure()
    assert g["n_leaves"] == e["n_leaves"] and g["height"] == e["height"]
    for f in ("level_sizes", "piv_key", "piv_id", "leaf_cnt", "leaf_lo", "leaf_hi", "node_lo", "node_hi",
              "node_cnt"):
        np.testing.assert_array_equal(g[f], e[f], err_msg=f)
    for a, b in zip(ix.export(), ref.dump()):
        np.testing.assert_array_equal(a, b)
    assert ix.size() == n


@pytest.mark.parametrize("B", [2, 3, 32])
def test_build_fanouts_and_leaf_sizes(psi, B):
    say(f"build fanout={B}")
    pts = synth.varden(50_000, 2, 30, seed=B)
    for phi in (4, 17, 32):
        ix, ref = make_pair(psi, 2, 1, pts, phi=phi, B=B)
        g, e = ix.structure(), ref.structure()
        for f in ("level_sizes", "piv_key", "piv_id", "leaf_cnt", "leaf_lo", "leaf_hi", "node_lo", "node_hi",
                  "node_cnt"):
            np.testing.assert_array_equal(g[f], e[f], err_msg=f"{f} phi={phi}")


def test_build_duplicates_heavy(psi):
    say("build duplicates")
    pts = synth.uniform(60_000, 3, 3, seed=5)  # 512 distinct points
    ix, ref = make_pair(psi, 3, 1, pts)
    for a, b in zip(ix.export(), ref.dump()):
        np.testing.assert_array_equal(a, b)
    g, e = ix.structure(), ref.structure()
    np.testing.assert_array_equal(g["piv_id"], e["piv_id"])


def test_build_out_of_range_latched(psi):
    say("build range error")
    pts = synth.uniform(1000, 3, 21, seed=1)
    pts[500, 0] = 1 << 21
    ix = psi.Index(3, 1)
    ix.build(pts)
    with pytest.raises(psi.PsiError) as e:
        ix.sync()
    assert e.value.code == 2
    ix.build(synth.uniform(10, 3, 21, seed=2))
    ix.sync()
    assert ix.size() == 10


def test_build_deterministic(psi):
    say("build determinism")
    pts = synth.varden(120_000, 3, 21, seed=8)
    a = psi.Index(3, 1).build(pts)
    b = psi.Index(3, 1).build(pts)
    sa, sb = a.structure(), b.structure()
    for f in sa:
        np.testing.assert_array_equal(np.asarray(sa[f]), np.asarray(sb[f]))
    for x, y in zip(a.leaves(), b.leaves()):
        np.testing.assert_array_equal(x, y)


# --------------------------------------------------------------------- kNN
@pytest.mark.parametrize("variant", [0, 2])
@pytest.mark.parametrize("k", [1, 10, 16, 17, 50, 100, 128])
@pytest.mark.parametrize("dim,curve", [(2, 1), (3, 1), (3, 0)])
def test_knn_parity(psi, dim, curve, k, variant):
    say(f"knn dim={dim} curve={curve} k={k} flags={variant}")
    data, _, q = synth.workload("varden", dim, bits_of(dim), seed=k, n=60_000, n_query=5000)
    ix = psi.Index(dim, curve, 32, 8, flags=variant).build(data)
    ref = oracle.RefIndex(dim, curve, 32, 8)
    ref.build(data)
    ids, d2 = ix.knn(q, k)
    eids, ed2 = ref.knn(q, k)
    np.testing.assert_array_equal(psi.to_u64(d2), ed2)
    np.testing.assert_array_equal(psi.to_u32(ids), eids)


@pytest.mark.parametrize("k", [3, 10, 40])
def test_knn_ties_small_domain(psi, k):
    # 4-bit coordinates: thousands of exact distance ties, decided by id
    say(f"knn ties k={k}")
    pts = synth.uniform(20_000, 2, 4, seed=k)
    q = synth.uniform(700, 2, 4, seed=k, purpose=synth.P_QUERY)
    ix, ref = make_pair(psi, 2, 1, pts, phi=8, B=4)
    alt = psi.Index(2, 1, 8, 4, flags=psi.FLAG_KNN_NEAREST_FIRST).build(pts)
    eids, ed2 = ref.knn(q, k)
    for g in (ix, alt):
        ids, d2 = g.knn(q, k)
        np.testing.assert_array_equal(psi.to_u64(d2), ed2)
        np.testing.assert_array_equal(psi.to_u32(ids), eids)


def test_knn_full_width_2d(psi):
    say("knn full-width 2d")
    pts = synth.uniform(30_000, 2, 31, seed=77)
    corners = np.array([[0, 0], [2**31 - 1, 2**31 - 1], [0, 2**31 - 1], [2**31 - 1, 0]], np.uint32)
    pts = np.concatenate([pts, corners])
    q = np.concatenate([corners, synth.uniform(300, 2, 31, seed=78)])
    ix, ref = make_pair(psi, 2, 0, pts)
    for k in (5, 33):
        ids, d2 = ix.knn(q, k)
        eids, ed2 = ref.knn(q, k)
        np.testing.assert_array_equal(psi.to_u64(d2), ed2)
        np.testing.assert_array_equal(psi.to_u32(ids), eids)


@pytest.mark.parametrize("n", [0, 1, 5, 40])
def test_knn_k_exceeds_n(psi, n):
    say(f"knn small n={n}")
    pts = synth.uniform(n, 3, 21, seed=n)
    q = synth.uniform(20, 3, 21, seed=n, purpose=synth.P_QUERY)
    ix, ref = make_pair(psi, 3, 1, pts, phi=4, B=2)
    for k in (8, 60):
        ids, d2 = ix.knn(q, k)
        eids, ed2 = ref.knn(q, k)
        np.testing.assert_array_equal(psi.to_u64(d2), ed2)
        np.testing.assert_array_equal(psi.to_u32(ids), eids)


@pytest.mark.parametrize("k", [10, 50])
def test_knn_walk_counts(psi, k):
    """The kNN walk counters: counting leaves the results unchanged; every
    query is counted once; a search reads at least the root's box, scans at
    least one leaf and at least k points (n > k), and never more points than
    its leaves hold (2 phi each) or than the index holds."""
    say(f"knn walk counts k={k}")
    n = 200_000
    data, _, q = synth.workload("uniform", 3, 21, seed=5, n=n, n_query=3000)
    ix = psi.Index(3, 1, 32, 8).build(data)
    ids0, d0 = ix.knn(q, k)
    assert not psi.psi_query_stats(ix._h, True).any()  # was off: zeros
    ids1, d1 = ix.knn(q, k)
    c = psi.psi_query_stats(ix._h, False).astype(np.int64)
    np.testing.assert_array_equal(psi.to_u32(ids0), psi.to_u32(ids1))
    np.testing.assert_array_equal(psi.to_u64(d0), psi.to_u64(d1))
    nq = len(q)
    assert c[0] == nq
    assert c[1] >= nq and c[2] >= nq
    assert k * nq <= c[3] <= min(64 * c[2], n * nq)
    say(f"  per query: {c[1] / nq:.1f} box tests, {c[2] / nq:.2f} leaves, {c[3] / nq:.1f} points")


# ------------------------------------------------------------------- range
@pytest.mark.parametrize("dim,curve", CURVES)
def test_range_parity(psi, dim, curve):
    say(f"range dim={dim} curve={curve}")
    bits = bits_of(dim)
    data, _, q = synth.workload("varden", dim, bits, seed=31, n=80_000, n_query=5000)
    bx = synth.boxes(q, bits, seed=32, side_lo=8, side_hi=22 if dim == 2 else 16)
    ix, ref = make_pair(psi, dim, curve, data)
    cnt = psi.to_u64(ix.range_count(bx))
    np.testing.assert_array_equal(cnt, ref.range_count(bx))
    off, ids = ix.range_report(bx)
    off = psi.to_u64(off)
    ids = psi.to_u32(ids)
    eoff, eids = ref.range_report(bx)
    np.testing.assert_array_equal(off, eoff)
    got = np.concatenate([np.sort(ids[off[b]:off[b + 1]]) for b in range(len(bx))]) if len(ids) else ids
    np.testing.assert_array_equal(got, eids)


def test_range_edge_boxes(psi):
    say("range edges")
    pts = synth.uniform(20_000, 3, 21, seed=9)
    ix, ref = make_pair(psi, 3, 1, pts)
    full = np.array([[[0, 0, 0], [2**21 - 1] * 3]], np.uint32)
    empty = np.array([[[5, 5, 5], [4, 9, 9]]], np.uint32)
    point = np.array([[pts[17], pts[17]]], np.uint32)
    bx = np.concatenate([full, empty, point])
    cnt = psi.to_u64(ix.range_count(bx))
    assert cnt[0] == 20_000 and cnt[1] == 0 and cnt[2] >= 1
    np.testing.assert_array_equal(cnt, ref.range_count(bx))
    off, ids = ix.range_report(bx)
    assert np.array_equal(np.sort(psi.to_u32(ids)[:20_000]), np.arange(20_000, dtype=np.uint32))


@pytest.mark.parametrize("dim,curve", [(2, 0), (3, 1)])
def test_query_order_is_invisible(psi, dim, curve):
    # batches of >= 4096 queries are processed in curve order; the results
    # must equal input-order processing and the oracle
    say(f"query order dim={dim} curve={curve}")
    bits = bits_of(dim)
    data, _, q = synth.workload("uniform", dim, bits, seed=41, n=200_000, n_query=20_000)
    a = psi.Index(dim, curve).build(data)
    b = psi.Index(dim, curve, flags=psi.FLAG_INPUT_ORDER).build(data)
    for k in (4, 24):
        ia, da = a.knn(q, k)
        ib, db = b.knn(q, k)
        np.testing.assert_array_equal(psi.to_u32(ia), psi.to_u32(ib))
        np.testing.assert_array_equal(psi.to_u64(da), psi.to_u64(db))
        sample = synth.sample_rows(len(q), 300, seed=k)
        eids, ed2 = oracle.knn_points(data, q[sample], k)
        np.testing.assert_array_equal(psi.to_u32(ia)[sample], eids)
        np.testing.assert_array_equal(psi.to_u64(da)[sample], ed2)
    bx = synth.boxes(q[:6000], bits, seed=42, side_lo=8, side_hi=20 if dim == 2 else 15)
    ca, cb = psi.to_u64(a.range_count(bx)), psi.to_u64(b.range_count(bx))
    np.testing.assert_array_equal(ca, cb)
    np.testing.assert_array_equal(ca[:500], oracle.range_count_points(data, bx[:500]))
    oa, ra = a.range_report(bx)
    ob, rb = b.range_report(bx)
    oa, ra, rb = psi.to_u64(oa), psi.to_u32(ra), psi.to_u32(rb)
    for i in range(0, len(bx), 97):
        np.testing.assert_array_equal(np.sort(ra[oa[i]:oa[i + 1]]), np.sort(rb[oa[i]:oa[i + 1]]))


@pytest.mark.parametrize("B,phi,n", [(2, 4, 3000), (3, 7, 5000), (32, 32, 70_000), (8, 32, 20)])
def test_range_fanouts(psi, B, phi, n):
    say(f"range fanout B={B} phi={phi} n={n}")
    pts = synth.varden(n, 3, 21, seed=B)
    ix, ref = make_pair(psi, 3, 1, pts, phi=phi, B=B)
    bx = synth.boxes(synth.varden(700, 3, 21, seed=B + 1), 21, seed=B + 2, side_lo=4, side_hi=20)
    np.testing.assert_array_equal(psi.to_u64(ix.range_count(bx)), ref.range_count(bx))
    off, ids = ix.range_report(bx)
    off, ids = psi.to_u64(off), psi.to_u32(ids)
    eoff, eids = ref.range_report(bx)
    np.testing.assert_array_equal(off, eoff)
    got = np.concatenate([np.sort(ids[off[b]:off[b + 1]]) for b in range(len(bx))])
    np.testing.assert_array_equal(got, eids)
