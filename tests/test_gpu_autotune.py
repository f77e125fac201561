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
    assert not r["cached"] and len(r["candidates"]) == 4
    assert (r["leaf_size"], r["fanout"], r["flags"]) in cands
    r2 = autotune.tune(3, 1, data, q, k=10, boxes=bx, candidates=cands, cache_path=cache)
    assert r2["cached"] and r2["leaf_size"] == r["leaf_size"]
    ix = psi.Index(3, 1, r["leaf_size"], r["fanout"], flags=r["flags"]).build(data)
    ids, d2 = ix.knn(q[:300], 10)
    ref = oracle.RefIndex(3, 1)
    ref.build(data)
    e_ids, e_d2 = ref.knn(q[:300], 10)
    np.testing.assert_array_equal(psi.to_u32(ids), e_ids)
    np.testing.assert_array_equal(psi.to_u64(d2), e_d2)
