"""hipGraph capture of query steps: every replay equals the eager result,
with the program's own eager work and synchronizations between replays.
(Captured builds and updates: test_gpu_enqueue.py.)"""
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


@pytest.mark.parametrize("nq", [777, 9000])  # 9000 >= 4096: the query sort runs inside the graph
def test_graph_replays_knn_and_range(psi, nq):
    import torch
    say(f"graph nq={nq}")
    stream = torch.cuda.Stream()
    dev = torch.device("cuda")
    data, _, q = synth.workload("uniform", 3, 21, seed=3, n=150_000, n_query=nq)
    bx = synth.boxes(q, 21, seed=4, side_lo=8, side_hi=16)
    with torch.cuda.stream(stream):
        ix = psi.Index(3, 1, 32, 8, device=dev, stream=stream)
        ix.build(data)
        h = ix._h
        dq = torch.from_numpy(q.view(np.int32)).to(dev)
        db = torch.from_numpy(bx.view(np.int32)).to(dev)
        ids = torch.empty((nq, 10), dtype=torch.int32, device=dev)
        d2 = torch.empty((nq, 10), dtype=torch.int64, device=dev)
        cnt = torch.empty(nq, dtype=torch.int64, device=dev)
        # eager reference (also sizes every buffer the capture will use)
        psi.psi_knn(h, dq, nq, 10, ids, d2)
        psi.psi_range_count(h, db, nq, cnt)
        stream.synchronize()
        e_ids, e_d2, e_cnt = ids.clone(), d2.clone(), cnt.clone()
        psi.psi_graph_begin(stream)
        psi.psi_knn(h, dq, nq, 10, ids, d2)
        psi.psi_range_count(h, db, nq, cnt)
        g = psi.psi_graph_end(stream)
        for rep in range(4):
            ids.fill_(-1)
            d2.fill_(-1)
            cnt.fill_(-1)
            psi.psi_graph_launch(g, stream)
            stream.synchronize()
            assert torch.equal(ids, e_ids) and torch.equal(d2, e_d2) and torch.equal(cnt, e_cnt), rep
            # eager work between replays, on the same index
            q2 = torch.from_numpy(synth.uniform(500, 3, 21, seed=rep, purpose=synth.P_AUX).view(np.int32)).to(dev)
            i2 = torch.empty((500, 4), dtype=torch.int32, device=dev)
            x2 = torch.empty((500, 4), dtype=torch.int64, device=dev)
            psi.psi_knn(h, q2, 500, 4, i2, x2)
            stream.synchronize()
        psi.psi_graph_destroy(g)
        ref = oracle.RefIndex(3, 1, 32, 8)
        ref.build(data)
        rows = synth.sample_rows(nq, 200, seed=5)
        r_ids, r_d2 = ref.knn(q[rows], 10)
        np.testing.assert_array_equal(psi.to_u32(e_ids)[rows], r_ids)
        np.testing.assert_array_equal(psi.to_u64(e_d2)[rows], r_d2)
        ix.sync()


def test_graph_multi_knn(psi):
    import torch
    say("graph multi knn")
    stream = torch.cuda.Stream()
    dev = torch.device("cuda")
    sizes = [5000, 1, 0, 40_000, 777]
    qsizes = [100, 3, 7, 2000, 0]
    pts = np.concatenate([synth.uniform(n, 2, 30, seed=10 + i) for i, n in enumerate(sizes)])
    qs = np.concatenate([synth.uniform(n, 2, 30, seed=20 + i) for i, n in enumerate(qsizes)])
    off = np.concatenate(([0], np.cumsum(sizes))).astype(np.uint64)
    qoff = np.concatenate(([0], np.cumsum(qsizes))).astype(np.uint64)
    with torch.cuda.stream(stream):
        M = psi.MultiIndex(2, 0, off, pts)
        dq = torch.from_numpy(qs.view(np.int32)).to(dev)
        dqo = torch.from_numpy(qoff.view(np.int64)).to(dev)
        ids = torch.empty((len(qs), 8), dtype=torch.int32, device=dev)
        d2 = torch.empty((len(qs), 8), dtype=torch.int64, device=dev)
        psi.psi_multi_knn(M._h, dqo, dq, 8, ids, d2)
        stream.synchronize()
        e_ids, e_d2 = ids.clone(), d2.clone()
        psi.psi_graph_begin(stream)
        psi.psi_multi_knn(M._h, dqo, dq, 8, ids, d2)
        g = psi.psi_graph_end(stream)
        for rep in range(3):
            ids.zero_()
            d2.zero_()
            psi.psi_graph_launch(g, stream)
            stream.synchronize()
            assert torch.equal(ids, e_ids) and torch.equal(d2, e_d2)
        psi.psi_graph_destroy(g)
        M.sync()
