"""Kernel timing (psi_prof_*): the families a build and a kNN pass bracket,
the restriction to one family (psi_prof_only), and results that do not
depend on whether timing is on.
"""
import sys

import numpy as np
import pytest

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


def test_one_family_timing(psi):
    say("timing: all families, then one family")
    pts = synth.uniform(200_003, 3, 21, seed=81)
    q = synth.uniform(5_000, 3, 21, seed=82, purpose=synth.P_QUERY)
    ix = psi.Index(3, 1, 32, 8)
    ix.build(pts)
    ids0, d20 = ix.knn(q, 10)
    ref_ids, ref_d2 = psi.to_u32(ids0), psi.to_u64(d20)

    ix.prof_enable(True)
    ix.prof_reset()
    ix.build(pts)
    ids, d2 = ix.knn(q, 10)
    knn_ms, knn_n, _ = ix.prof_get("knn")
    fill_ms, fill_n, fill_b = ix.prof_get("leaf_fill")
    assert knn_n >= 1 and knn_ms > 0
    assert fill_n >= 1 and fill_ms > 0 and fill_b > 0
    np.testing.assert_array_equal(psi.to_u32(ids), ref_ids)
    np.testing.assert_array_equal(psi.to_u64(d2), ref_d2)

    ix.prof_only("knn")
    ix.prof_reset()
    ix.build(pts)
    ids, d2 = ix.knn(q, 10)
    assert ix.prof_get("knn")[1] >= 1
    assert ix.prof_get("leaf_fill") == (0.0, 0, 0)
    np.testing.assert_array_equal(psi.to_u32(ids), ref_ids)
    np.testing.assert_array_equal(psi.to_u64(d2), ref_d2)

    ix.prof_only(None)
    ix.prof_reset()
    ix.build(pts)
    assert ix.prof_get("leaf_fill")[1] >= 1
    ix.prof_enable(False)
    ix.prof_reset()
    ix.build(pts)
    assert ix.prof_get("leaf_fill") == (0.0, 0, 0)
    ix.sync()
