"""GPU parity of the paper's incremental-update workload (Sec. 5.1): an index
built from empty by n/b batch insertions, then emptied by n/b batch deletions,
with kNN queries after half of the insertion batches and after half of the
deletion batches, in- and out-of-distribution. After every batch the set,
the ids and (at the checkpoints) the structure invariants and query results
equal the oracle's; at the insertion checkpoint the kNN answers also equal
those of a static build of the same points (same ids, since ids are assigned
in insertion order).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from invariants import check

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


def bits_of(dim):
    return 30 if dim == 2 else 21


def queries(dist, nq, dim, bits, seed):
    """In-distribution queries (a separate draw of the data's law) and
    out-of-distribution ones (varden queries for uniform and sweepline data,
    uniform ones for varden data)."""
    ind = synth.points("uniform" if dist == "sweepline" else dist, nq, dim, bits, seed, synth.P_QUERY)
    ood = synth.points("uniform" if dist == "varden" else "varden", nq, dim, bits, seed + 1, synth.P_QUERY)
    return ind, ood


def knn_equal(psi, ix, ref, q, k):
    ids, d2 = ix.knn(q, k)
    eids, ed2 = ref.knn(q, k)
    np.testing.assert_array_equal(psi.to_u64(d2), ed2)
    np.testing.assert_array_equal(psi.to_u32(ids), eids)
    return psi.to_u32(ids)


@pytest.mark.parametrize("dist", ["sweepline", "uniform", "varden"])
@pytest.mark.parametrize("dim,curve,frac", [(2, 0, 0.02), (3, 1, 0.05), (2, 1, 0.1)])
def test_incremental_build_and_empty(psi, dist, dim, curve, frac):
    n, phi, B, k = 24_000, 32, 8, 10
    bits = bits_of(dim)
    say(f"incremental dist={dist} dim={dim} curve={curve} b={frac}")
    pts = synth.points(dist, n, dim, bits, seed=61)
    ind, ood = queries(dist, 400, dim, bits, seed=62)
    s = int(n * frac)
    nbat = n // s
    ix = psi.Index(dim, curve, phi, B).build(np.zeros((0, dim), np.uint32))
    ref = oracle.RefIndex(dim, curve, phi, B)
    ref.build(np.zeros((0, dim), np.uint32))
    for i in range(nbat):
        batch = pts[i * s:(i + 1) * s]
        np.testing.assert_array_equal(psi.to_u32(ix.batch_insert(batch)), ref.batch_insert(batch))
        if i == nbat // 2 - 1:  # half of the insertion batches
            ix.sync()
            for a, b in zip(ix.export(), ref.dump()):
                np.testing.assert_array_equal(a, b)
            check(ix, phi, B, curve)
            static = psi.Index(dim, curve, phi, B).build(pts[:(i + 1) * s])
            for q in (ind, ood):
                got = knn_equal(psi, ix, ref, q, k)
                np.testing.assert_array_equal(got, psi.to_u32(static.knn(q, k)[0]))
            static.sync()
    ix.sync()
    assert ix.size() == ref.size() == nbat * s
    for a, b in zip(ix.export(), ref.dump()):
        np.testing.assert_array_equal(a, b)
    check(ix, phi, B, curve)
    for i in range(nbat):  # deletion in insertion order: batch i removes ids [i s, (i + 1) s)
        ids = np.arange(i * s, (i + 1) * s, dtype=np.uint32)
        assert int(psi.to_u64(ix.batch_delete(ids))[0]) == ref.batch_delete(ids) == s
        if i == nbat // 2 - 1:  # half of the deletion batches
            ix.sync()
            for a, b in zip(ix.export(), ref.dump()):
                np.testing.assert_array_equal(a, b)
            check(ix, phi, B, curve)
            for q in (ind, ood):
                knn_equal(psi, ix, ref, q, k)
    ix.sync()
    assert ix.size() == ref.size() == 0
    ids, d2 = ix.knn(ind[:5], 3)
    assert (psi.to_u32(ids) == 0xFFFFFFFF).all() and (psi.to_u64(d2) == np.iinfo(np.uint64).max).all()
