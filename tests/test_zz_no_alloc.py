"""The allocation-free sort (psi_sort_pairs_noalloc) against the allocating
one (psi_sort_pairs) and numpy's lexsort, on calls in a row through the same
per-GPU workspace, each smaller than the one before."""
import sys

import numpy as np
import pytest

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


def _pairs(n, seed):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 1 << 40, size=n, dtype=np.uint64)
    keys[: n // 3] = keys[n // 3: 2 * (n // 3)]  # many equal keys: their ids decide
    ids = rng.permutation(np.arange(n, dtype=np.uint64) * 7 + 3).astype(np.uint32)
    return keys, ids


def test_noalloc_sort_equals_the_allocating_sort(psi):
    import torch
    dev = torch.device("cuda")
    for rnd, n in enumerate([psi.SORT_NOALLOC_MAX, 300_000, 70_001, 9_000, 1]):
        say(f"noalloc sort n={n}")
        keys, ids = _pairs(n, seed=100 + rnd)
        dk = torch.from_numpy(keys.view(np.int64)).to(dev)
        di = torch.from_numpy(ids.view(np.int32)).to(dev)
        ka, ia = torch.empty_like(dk), torch.empty_like(di)
        kb, ib = torch.empty_like(dk), torch.empty_like(di)
        psi.psi_sort_pairs_noalloc(dk, di, n, ka, ia)
        psi.psi_sort_pairs(dk, di, n, kb, ib)
        torch.cuda.synchronize()
        assert torch.equal(ka, kb) and torch.equal(ia, ib), n
        o = np.lexsort((ids, keys))
        np.testing.assert_array_equal(psi.to_u64(ka), keys[o])
        np.testing.assert_array_equal(psi.to_u32(ia), ids[o])
        # the inputs are left as they were
        np.testing.assert_array_equal(psi.to_u64(dk), keys)


def test_noalloc_sort_refuses_more_than_its_workspace(psi):
    import torch
    dev = torch.device("cuda")
    n = psi.SORT_NOALLOC_MAX + 1
    dk = torch.zeros(n, dtype=torch.int64, device=dev)
    di = torch.zeros(n, dtype=torch.int32, device=dev)
    with pytest.raises(psi.PsiError) as e:
        psi.psi_sort_pairs_noalloc(dk, di, n, dk.clone(), di.clone())
    assert e.value.code == 1
