"""The autotuner returns a valid configuration, every candidate gives the same
answers (checked inside the tuner), and the chosen configuration is exact
against the oracle."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_autotune_small(tmp_path):
    import torch
    assert torch.cuda.is_available()
    import paper_2601_05347_amd as psi
    from paper_2601_05347_amd import autotune
    data, _, q = synth.workload("varden", 3, 21, seed=9, n=200_000, n_query=20_000)
    bx = synth.boxes(q[:5000], 21, seed=10, side_lo=8, side_hi=15)
    cache = str(tmp_path / "tune.json")
    cands = [(16, 4, 0), (32, 8, 0), (32, 8, psi.FLAG_KNN_NEAREST_FIRST), (24, 16, psi.FLAG_INPUT_ORDER)]
    r = autotune.tune(3, 1, data, q, k=10, boxes=bx, candidates=cands, cache_path=cache)
    assert not r["cached"]
    stages = [c["stage"] for c in r["candidates"]]
    assert stages.count("structure") == 4 and stages.count("order") == 4 and stages.count("build_sort") == 3
    if not (r["flags"] & psi.FLAG_KNN_NEAREST_FIRST):
        assert stages.count("knn_walk") == len(autotune.SEED_LEAVES) * len(autotune.CAND_LENGTHS)
    base = r["flags"] & ~(psi.FLAG_INPUT_ORDER | psi.FLAG_SORT_BUCKETS | psi.FLAG_SORT_LSD)
    assert any((r["leaf_size"], r["fanout"]) == c[:2] and base == c[2] & ~psi.FLAG_INPUT_ORDER for c in cands)
    t = r["tuning"]
    assert t["knn_seed_leaves"] in autotune.SEED_LEAVES and t["knn_cand"] in autotune.CAND_LENGTHS
    assert t["order_bits"] in autotune.ORDER_BITS
    r2 = autotune.tune(3, 1, data, q, k=10, boxes=bx, candidates=cands, cache_path=cache)
    assert r2["cached"] and r2["leaf_size"] == r["leaf_size"] and r2["tuning"] == t
    ix = psi.Index(3, 1, r["leaf_size"], r["fanout"], flags=r["flags"]).build(data)
    autotune.apply(ix, r)
    assert psi.psi_get_tuning(ix._h) == t
    ids, d2 = ix.knn(q[:300], 10)
    ref = oracle.RefIndex(3, 1)
    ref.build(data)
    e_ids, e_d2 = ref.knn(q[:300], 10)
    np.testing.assert_array_equal(psi.to_u32(ids), e_ids)
    np.testing.assert_array_equal(psi.to_u64(d2), e_d2)


def test_tuning_knobs_checked_and_exact():
    """psi_set_tuning rejects values out of range (and keeps the old ones);
    every accepted setting gives the oracle's answers."""
    import torch
    assert torch.cuda.is_available()
    import paper_2601_05347_amd as psi
    data, _, q = synth.workload("uniform", 2, 30, seed=4, n=120_000, n_query=6000)
    ix = psi.Index(2, 1, 32, 8).build(data)
    for bad in ({"knn_seed_leaves": 2}, {"knn_seed_leaves": 11}, {"knn_cand": 0}, {"knn_cand": 33},
                {"order_bits": 12}, {"order_bits": 40}):
        with pytest.raises(psi.PsiError) as e:
            psi.psi_set_tuning(ix._h, **bad)
        assert e.value.code == 1
    assert psi.psi_get_tuning(ix._h) == {"knn_seed_leaves": 3, "knn_cand": 16, "order_bits": 24}
    ref = oracle.RefIndex(2, 1)
    ref.build(data)
    e_ids, e_d2 = ref.knn(q, 8)
    for s_, c_, b_ in ((1, 1, 8), (9, 32, 32), (5, 4, 16)):
        psi.psi_set_tuning(ix._h, knn_seed_leaves=s_, knn_cand=c_, order_bits=b_)
        ids, d2 = ix.knn(q, 8)
        np.testing.assert_array_equal(psi.to_u32(ids), e_ids)
        np.testing.assert_array_equal(psi.to_u64(d2), e_d2)
