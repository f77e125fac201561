"""GPU parity of the two-level build sort (top-bit buckets, then per-bucket
LDS sort; oversized buckets through segmented global passes) against the
oracle, and against the eight-pass LSD build, bit-exact.

Bucket = the 16 key bits below the largest key's leading bit. With 2D Morton
keys and a largest coordinate of 2^31 - 1 those are bits 23..30 of both
coordinates, which lets the tests place exact bucket sizes: 2048 (the largest
the light LDS variant sorts), 2049 (the smallest the wide variant takes), 4096
(the largest the wide variant sorts), 4097 and 8192 (the smallest and largest
the 1024-thread variant takes) and 8193 (the smallest that takes the
segmented global passes).
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CURVES = [(2, 0), (2, 1), (3, 0), (3, 1)]
FIELDS = ("level_sizes", "piv_key", "piv_id", "leaf_cnt", "leaf_lo", "leaf_hi", "node_lo", "node_hi", "node_cnt")


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


def check(psi, dim, curve, pts, phi=32, B=8):
    """Two-level build == oracle (structure, sorted dump) == LSD build (raw leaves)."""
    ix = psi.Index(dim, curve, phi, B, flags=psi.FLAG_SORT_BUCKETS).build(pts)
    ref = oracle.RefIndex(dim, curve, phi, B)
    ref.build(pts)
    g, e = ix.structure(), ref.structure()
    assert g["n_leaves"] == e["n_leaves"] and g["height"] == e["height"]
    for f in FIELDS:
        np.testing.assert_array_equal(g[f], e[f], err_msg=f)
    for a, b in zip(ix.export(), ref.dump()):
        np.testing.assert_array_equal(a, b)
    lsd = psi.Index(dim, curve, phi, B, flags=psi.FLAG_SORT_LSD).build(pts)
    for a, b in zip(ix.leaves(), lsd.leaves()):
        np.testing.assert_array_equal(a, b)
    ix.sync()
    lsd.sync()
    return ix, ref


@pytest.mark.parametrize("n", [1, 33, 4097, 100_003, 1_000_003])
@pytest.mark.parametrize("dim,curve", CURVES)
def test_two_level_uniform(psi, dim, curve, n):
    say(f"two-level uniform dim={dim} curve={curve} n={n}")
    check(psi, dim, curve, synth.uniform(n, dim, bits_of(dim), seed=n + 11))


def test_bucket_size_boundaries(psi):
    """Buckets of exactly 2048, 2049, 4096 and 4097 pairs, an empty bucket
    between them, a bucket of 1 and a uniform remainder (2D Morton: bucket
    bit j is bit 23 + j // 2 of axis j % 2)."""
    say("two-level bucket boundaries")
    sizes = [(2048, (1, 0)), (2049, (0, 1)), (4096, (1, 1)), (4097, (2, 0)), (1, (0, 3)), (8192, (3, 0)),
             (8193, (0, 2))]
    rest = 50_000
    r = synth.uniform(sum(c for c, _ in sizes) + rest, 2, 23, seed=3)  # low 23 bits of each coordinate
    hi = np.zeros((len(r), 2), np.uint32)
    o = 0
    for c, (hx, hy) in sizes:  # buckets 1, 2, 3, 4 and 10
        hi[o:o + c, 0] = hx
        hi[o:o + c, 1] = hy
        o += c
    hi[o:, 0] = synth.uniform(rest, 1, 8, seed=4)[:, 0]
    hi[o:, 1] = synth.uniform(rest, 1, 8, seed=5)[:, 0] | 4  # bucket bit 5 set: never one of the above
    hi[-1] = (255, 255)  # the largest coordinates: key bit length 62 (buckets 5 and 8 above)
    pts = (r | (hi << np.uint32(23))).astype(np.uint32)
    perm = np.argsort(synth.draws(synth.stream_key(9, synth.P_AUX), 0, len(pts)), kind="stable")
    check(psi, 2, 0, pts[perm])


@pytest.mark.parametrize("dim,curve", [(2, 0), (3, 1)])
def test_single_big_bucket(psi, dim, curve):
    """Every key in one bucket: the whole sort runs in the segmented passes."""
    say(f"two-level one big bucket dim={dim} curve={curve}")
    check(psi, dim, curve, synth.uniform(300_007, dim, 12 if dim == 2 else 8, seed=7))


def test_mixed_big_and_small_buckets(psi):
    say("two-level mixed buckets")
    a = synth.uniform(200_000, 3, 21, seed=12)
    b = synth.uniform(150_000, 3, 6, seed=13) + np.uint32(1 << 20)  # one dense corner cell
    pts = np.concatenate([a, b]).astype(np.uint32)
    check(psi, 3, 1, pts[np.argsort(synth.draws(synth.stream_key(14, synth.P_AUX), 0, len(pts)), kind="stable")])


def test_clustered_varden(psi):
    say("two-level varden 2D/3D")
    check(psi, 2, 1, synth.varden(1_000_000, 2, 30, seed=21))
    check(psi, 3, 0, synth.varden(1_000_000, 3, 21, seed=22))


def test_equal_keys_keep_id_order(psi):
    """Equal keys (duplicate points) stay in id order, in small and big buckets."""
    say("two-level duplicates")
    check(psi, 3, 1, synth.uniform(60_000, 3, 3, seed=5))  # 512 distinct points
    same = np.tile(np.array([[123456, 7654321]], np.uint32), (20_000, 1))
    check(psi, 2, 1, same)


def test_fanouts_leaf_sizes_and_updates(psi):
    say("two-level phi/B and updates")
    pts = synth.varden(80_000, 2, 30, seed=31)
    for phi, B in ((4, 2), (17, 3), (32, 32)):
        check(psi, 2, 1, pts, phi=phi, B=B)
    ix, ref = check(psi, 3, 1, synth.uniform(120_000, 3, 21, seed=32))
    ins = synth.uniform(5000, 3, 21, seed=33, purpose=synth.P_INSERT)
    np.testing.assert_array_equal(psi.to_u32(ix.batch_insert(ins)), ref.batch_insert(ins))
    dels = synth.delete_ids(np.arange(ref.next_id(), dtype=np.uint32), 7000, seed=34)
    assert int(psi.to_u64(ix.batch_delete(dels))[0]) == ref.batch_delete(dels)
    for a, b in zip(ix.export(), ref.dump()):
        np.testing.assert_array_equal(a, b)
    ix.sync()


def test_flags_validated(psi):
    with pytest.raises(psi.PsiError):
        psi.Index(2, 0, flags=psi.FLAG_SORT_BUCKETS | psi.FLAG_SORT_LSD)


def _bucket0(n_spread, n_cluster, cluster_bits, seed):
    """2D Morton points of bucket 0 (coordinates below 2^23): n_spread spread
    over the whole bucket, n_cluster inside [0, 2^cluster_bits)^2."""
    a = synth.uniform(n_spread, 2, 23, seed=seed)
    c = synth.uniform(n_cluster, 2, cluster_bits, seed=seed + 1)
    return np.concatenate([a, c])


def test_skewed_buckets(psi):
    """Sub-buckets of 17..32 pairs (ranked by a wave), buckets whose pairs
    crowd into one sub-bucket (the LDS LSD fallback of the wide variant: one
    above 2048 pairs, one below that the light variant hands over), and a
    bucket of equal keys, among uniform buckets."""
    say("two-level skewed buckets")
    rest = synth.uniform(200_000, 2, 31, seed=40)
    rest = rest[((rest[:, 0] >> 23) > 1) | ((rest[:, 1] >> 23) > 1)]  # keep buckets 0..3 for the parts below
    net32 = _bucket0(900, 20, 10, seed=41)                     # bucket 0
    crowd = _bucket0(12, 3000, 4, seed=43) | np.array([1 << 23, 0], np.uint32)   # bucket 1
    same = np.tile(np.array([[77, 1 << 23]], np.uint32), (2500, 1))            # bucket 2
    crowd_small = _bucket0(10, 1490, 4, seed=45) | np.array([1 << 23, 1 << 23], np.uint32)  # bucket 3
    pts = np.concatenate([rest, net32, crowd, same, crowd_small]).astype(np.uint32)
    pts = pts[np.argsort(synth.draws(synth.stream_key(44, synth.P_AUX), 0, len(pts)), kind="stable")]
    check(psi, 2, 0, pts)


def _axes_of_bucket(t):
    """(x >> 23, y >> 23) of the 2D Morton points in bucket t (bucket bit j
    is bit 23 + j // 2 of axis j % 2)."""
    hx = sum(((t >> (2 * i)) & 1) << i for i in range(8))
    hy = sum(((t >> (2 * i + 1)) & 1) << i for i in range(8))
    return hx, hy


def test_huge_buckets(psi):
    """Buckets of 4097..8192 pairs (the 1024-thread LDS variant): the two
    ends, more of them than that launch has workgroups (each loops over the
    list), a bucket of equal keys, a bucket whose pairs crowd into one
    sub-bucket (left to the segmented passes), one of 8193 pairs (the
    segmented passes), among small uniform buckets."""
    say("two-level huge buckets")
    draws = synth.draws(synth.stream_key(61, synth.P_AUX), 0, 300)
    sizes = [4097, 8192, 8193] + [4097 + int(d % 4096) for d in draws]
    parts, t = [], 0
    for i, c in enumerate(sizes):  # buckets 0 .. len(sizes) - 1
        low = synth.uniform(c, 2, 23, seed=100 + i)
        hx, hy = _axes_of_bucket(t)
        parts.append(low | np.array([hx << 23, hy << 23], np.uint32))
        t += 1
    hx, hy = _axes_of_bucket(t)  # equal keys
    parts.append(np.tile(np.array([[5 | (hx << 23), 9 | (hy << 23)]], np.uint32), (6000, 1)))
    t += 1
    hx, hy = _axes_of_bucket(t)  # 6900 pairs in 64 grid points, 100 spread: one sub-bucket of > 64
    crowd = np.concatenate([synth.uniform(6900, 2, 3, seed=70), synth.uniform(100, 2, 23, seed=71)])
    parts.append(crowd | np.array([hx << 23, hy << 23], np.uint32))
    t += 1
    rest = synth.uniform(50_000, 2, 23, seed=72)
    hb = 60_000 + synth.draws(synth.stream_key(73, synth.P_AUX), 0, len(rest)) % 5535
    hxy = np.array([_axes_of_bucket(int(b)) for b in hb], np.uint32)
    parts.append(rest | (hxy << np.uint32(23)))
    parts.append(np.array([[0x7FFFFFFF, 0x7FFFFFFF]], np.uint32))  # key bit length 62
    pts = np.concatenate(parts).astype(np.uint32)
    pts = pts[np.argsort(synth.draws(synth.stream_key(74, synth.P_AUX), 0, len(pts)), kind="stable")]
    check(psi, 2, 0, pts)


def test_rebuild_with_other_key_widths(psi):
    """One index rebuilt over data of different key widths: the bucket digits
    counted while encoding are for the previous build's bucket bits, right or
    wrong for the new data; the result is the same either way."""
    say("two-level rebuilds across key widths")
    ix = psi.Index(3, 1, 32, 8, flags=psi.FLAG_SORT_BUCKETS)
    for bits, seed in ((21, 51), (21, 52), (9, 53), (9, 54), (17, 55), (21, 56), (4, 57)):
        pts = synth.uniform(70_001, 3, bits, seed=seed)
        ix.build(pts)
        ref = oracle.RefIndex(3, 1, 32, 8)
        ref.build(pts)
        for a, b in zip(ix.export(), ref.dump()):
            np.testing.assert_array_equal(a, b)
    ix.sync()
