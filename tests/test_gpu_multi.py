"""Batched small indexes: one segmented build and one persistent kNN launch
over many independent indexes must give, for every index, exactly what the
oracle (and the single-index path) gives for that index alone."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


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


def batch(dim, sizes, qsizes, seed, bits=30):
    pts = [synth.uniform(int(n), dim, bits, seed=seed + i) for i, n in enumerate(sizes)]
    qs = [synth.uniform(int(n), dim, bits, seed=seed + i, purpose=synth.P_QUERY) for i, n in enumerate(qsizes)]
    off = np.concatenate(([0], np.cumsum(sizes))).astype(np.uint64)
    qoff = np.concatenate(([0], np.cumsum(qsizes))).astype(np.uint64)
    return pts, qs, off, qoff


@pytest.mark.parametrize("dim,curve", [(2, 0), (2, 1), (3, 1)])
def test_multi_matches_single(psi, dim, curve):
    say(f"multi dim={dim} curve={curve}")
    sizes = [0, 1, 31, 32, 33, 4095, 4096, 4097, 10_000, 25_000, 7, 0, 900]
    qsizes = [3, 0, 64, 65, 1, 200, 0, 130, 500, 640, 9, 5, 70]
    bits = 30 if dim == 2 else 21
    pts, qs, off, qoff = batch(dim, sizes, qsizes, seed=dim * 10 + curve, bits=bits)
    allp = np.concatenate(pts).reshape(-1, dim)
    allq = np.concatenate(qs).reshape(-1, dim)
    M = psi.MultiIndex(dim, curve, off, allp, 32, 8)
    k_all, i_all, p_all = M.export()
    for k in (8, 1, 16):
        ids, d2 = M.knn(qoff, allq, k)
        ids, d2 = psi.to_u32(ids), psi.to_u64(d2)
        for s, (p, q) in enumerate(zip(pts, qs)):
            ref = oracle.RefIndex(dim, curve, 32, 8)
            ref.build(p)
            a, b = int(qoff[s]), int(qoff[s + 1])
            if b > a:
                eids, ed2 = ref.knn(q, k)
                np.testing.assert_array_equal(d2[a:b], ed2, err_msg=f"index {s}")
                np.testing.assert_array_equal(ids[a:b], eids, err_msg=f"index {s}")
            if k == 8:
                g, e = M.structure(s), ref.structure()
                assert g["n_leaves"] == e["n_leaves"]
                for f in ("level_sizes", "piv_key", "piv_id", "leaf_cnt", "leaf_lo", "leaf_hi", "node_lo",
                          "node_hi", "node_cnt"):
                    np.testing.assert_array_equal(g[f], e[f], err_msg=f"{f} index {s}")
                lo, hi = int(off[s]), int(off[s + 1])
                ek, ei, ep = ref.dump()
                np.testing.assert_array_equal(k_all[lo:hi], ek)
                np.testing.assert_array_equal(i_all[lo:hi], ei)
                np.testing.assert_array_equal(p_all[lo:hi], ep)
    M.sync()


def test_multi_many_indexes(psi):
    # 300 indexes, sizes log-uniform in 1e2..3e4, uneven query batches
    say("multi many")
    r = synth.unit(synth.draws(synth.stream_key(5, 9), 0, 600))
    sizes = np.floor(10 ** (2 + 2.5 * r[:300])).astype(np.int64)
    qsizes = np.floor(10 ** (3 * r[300:])).astype(np.int64)
    pts, qs, off, qoff = batch(2, sizes, qsizes, seed=777)
    allp = np.concatenate(pts)
    allq = np.concatenate(qs)
    M = psi.MultiIndex(2, 0, off, allp, 32, 8)
    ids, d2 = M.knn(qoff, allq, 8)
    ids, d2 = psi.to_u32(ids), psi.to_u64(d2)
    single = psi.Index(2, 0, 32, 8)
    for s in range(0, 300, 7):
        a, b = int(qoff[s]), int(qoff[s + 1])
        single.build(pts[s])
        if b > a:
            gi, gd = single.knn(qs[s], 8)
            np.testing.assert_array_equal(d2[a:b], psi.to_u64(gd))
            np.testing.assert_array_equal(ids[a:b], psi.to_u32(gi))
            eids, ed2 = oracle.knn_points(pts[s], qs[s][:50], 8)
            np.testing.assert_array_equal(d2[a:a + min(50, b - a)], ed2[: b - a])
    M.sync()


def test_multi_rejects_bad_input(psi):
    say("multi errors")
    import torch
    pts = synth.uniform(100, 2, 30, seed=1)
    bad_off = np.array([0, 50, 40, 100], np.uint64)  # not monotone
    with pytest.raises(psi.PsiError) as e:
        psi.MultiIndex(2, 0, bad_off, pts)
    assert e.value.code == 1
    M = psi.MultiIndex(2, 0, np.array([0, 60, 100], np.uint64), pts)
    with pytest.raises(psi.PsiError):
        M.knn(np.array([0, 1, 2], np.uint64), pts[:2], 3)  # k = 3 unsupported here
    torch.cuda.synchronize()


def test_multi_full_size(psi):
    """The batched-index configuration at its real size: 4096 2D SPaC-Z
    indexes with sizes log-uniform in 1e3..1e6 (about 5.8e8 points) and
    1..1e4 queries each, k = 8. Every row is checked for what holds at any
    size (d2 equal to the squared distance to the returned point of its own
    index, rows ascending in (d2, id)); a seeded sample of indexes is
    brute-forced by the oracle."""
    import torch
    say("multi full size")
    num = 4096
    r = synth.unit(synth.draws(synth.stream_key(0, 77), 0, 2 * num))
    sizes = np.floor(10 ** (3 + 3 * r[:num])).astype(np.int64)
    qsizes = np.floor(10 ** (4 * r[num:])).astype(np.int64).clip(1, 10_000)
    allp = np.concatenate([synth.uniform(int(n), 2, 30, 1000 + i) for i, n in enumerate(sizes)])
    allq = np.concatenate([synth.uniform(int(n), 2, 30, 1000 + i, synth.P_QUERY) for i, n in enumerate(qsizes)])
    off = np.concatenate(([0], np.cumsum(sizes))).astype(np.uint64)
    qoff = np.concatenate(([0], np.cumsum(qsizes))).astype(np.uint64)
    say(f"  {len(allp)} points, {len(allq)} queries")
    M = psi.MultiIndex(2, 0, off, allp, 32, 8)
    ids, d2 = M.knn(qoff, allq, 8)
    M.sync()
    dev = ids.device
    owner = torch.repeat_interleave(torch.arange(num, device=dev), torch.from_numpy(qsizes).to(dev))
    base = torch.from_numpy(off[:-1].astype(np.int64)).to(dev)[owner]
    loc = ids.long()
    assert bool((loc >= 0).all()) and bool((loc < torch.from_numpy(sizes).to(dev)[owner].unsqueeze(1)).all())
    pts_d = torch.from_numpy(allp.astype(np.int64)).to(dev)
    q_d = torch.from_numpy(allq.astype(np.int64)).to(dev)
    for a in range(0, len(allq), 1_000_000):
        g = loc[a:a + 1_000_000] + base[a:a + 1_000_000].unsqueeze(1)
        dd = ((pts_d[g] - q_d[a:a + 1_000_000].unsqueeze(1)) ** 2).sum(-1)
        assert torch.equal(dd, d2[a:a + 1_000_000])
        l, d = loc[a:a + 1_000_000], d2[a:a + 1_000_000]
        assert bool(((d[:, :-1] < d[:, 1:]) | ((d[:, :-1] == d[:, 1:]) & (l[:, :-1] < l[:, 1:]))).all())
    del pts_d, q_d
    h_ids, h_d2 = psi.to_u32(ids), psi.to_u64(d2)
    for s in synth.sample_rows(num, 8, seed=78):
        a, b = int(qoff[s]), int(qoff[s + 1])
        rows = np.arange(a, b)[: 256]
        p = allp[int(off[s]):int(off[s + 1])]
        eids, ed2 = oracle.knn_points(p, allq[rows], 8, threads=16)
        np.testing.assert_array_equal(h_d2[rows], ed2, err_msg=f"index {s}")
        np.testing.assert_array_equal(h_ids[rows], eids, err_msg=f"index {s}")
