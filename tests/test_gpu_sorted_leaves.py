"""The total-order ablation (PSI_FLAG_SORTED_LEAVES): with the flag every
leaf holds its entries in (key, id) order after every update, as a
CPAM-style tree keeps them; without it inserts append unsorted (Sec. 4.2).
Both give the oracle's set and the oracle's query answers."""
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


def leaf_orders(ix, dim, curve):
    """Per leaf: whether its stored entries are in (key, id) order."""
    ids, pts = ix.leaves()
    cnt = ix.structure()["leaf_cnt"].astype(np.int64)
    keys = oracle.encode(pts, dim, curve)
    out, o = [], 0
    for c in cnt:
        k, i = keys[o:o + c], ids[o:o + c].astype(np.uint64)
        out.append(bool(np.all((k[1:] > k[:-1]) | ((k[1:] == k[:-1]) & (i[1:] > i[:-1])))))
        o += c
    return np.array(out)


@pytest.mark.parametrize("dim,curve", [(2, 0), (3, 1)])
def test_sorted_leaves_flag(psi, dim, curve):
    say(f"sorted leaves dim={dim} curve={curve}")
    bits = 30 if dim == 2 else 21
    data, ins, q = synth.workload("uniform", dim, bits, seed=81, n=40_000, n_insert=36_000, n_query=300)
    ix = psi.Index(dim, curve, 32, 8, flags=psi.FLAG_SORTED_LEAVES).build(data)
    plain = psi.Index(dim, curve, 32, 8).build(data)
    ref = oracle.RefIndex(dim, curve, 32, 8)
    ref.build(data)
    assert leaf_orders(ix, dim, curve).all()
    for b in range(4):  # appends, then re-cut leaves as the slots fill up
        batch = ins[b * 9000:(b + 1) * 9000]
        got = psi.to_u32(ix.batch_insert(batch))
        np.testing.assert_array_equal(got, ref.batch_insert(batch))
        plain.batch_insert(batch)
        ix.sync()
        assert leaf_orders(ix, dim, curve).all(), f"insert batch {b}"
        for a, e in zip(ix.export(), ref.dump()):
            np.testing.assert_array_equal(a, e)
    # without the flag the appended leaves are left in arrival order
    assert not leaf_orders(plain, dim, curve).all()
    dels = synth.delete_ids(np.arange(ref.next_id(), dtype=np.uint32), 50_000, seed=82)
    for b in range(2):  # deletes compact stably and regroup from sorted leaves
        d = dels[b * 25_000:(b + 1) * 25_000]
        assert int(psi.to_u64(ix.batch_delete(d))[0]) == ref.batch_delete(d)
        ix.sync()
        assert leaf_orders(ix, dim, curve).all(), f"delete batch {b}"
        for a, e in zip(ix.export(), ref.dump()):
            np.testing.assert_array_equal(a, e)
    ids, d2 = ix.knn(q, 10)
    eids, ed2 = ref.knn(q, 10)
    np.testing.assert_array_equal(psi.to_u64(d2), ed2)
    np.testing.assert_array_equal(psi.to_u32(ids), eids)
    plain.sync()
    ix.sync()
