"""MI355X (gfx950) SPaC-tree spatial index: Python binding of libpsi.so.

The binding only marshals arguments: every step of build, update and query
runs in the HIP kernels of libpsi.so. Device memory and streams come from
PyTorch (tensors on a ROCm device, `torch.cuda.current_stream()`). There is
no CPU fallback: if libpsi.so is missing or no GPU is present, calls raise.

Functions named psi_* mirror the C ABI in include/psi.h one to one; `Index`
is a small convenience wrapper that allocates the output tensors.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsi.so")

MORTON, HILBERT = 0, 1
FLAG_INPUT_ORDER = 1
FLAG_KNN_NEAREST_FIRST = 2
FLAG_SORT_BUCKETS = 4
FLAG_SORT_LSD = 8
FLAG_SORTED_LEAVES = 16
PAD_ID = 0xFFFFFFFF
PAD_D2 = 0xFFFFFFFFFFFFFFFF

STATUS = {0: "PSI_OK", 1: "PSI_E_ARG", 2: "PSI_E_RANGE", 3: "PSI_E_NOMEM", 4: "PSI_E_CAPACITY",
          5: "PSI_E_HIP", 6: "PSI_E_STATE", 7: "PSI_E_INTERNAL"}

# exported symbols of include/psi.h with (restype, argtypes)
_P, _u64, _u32, _i = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int
SIGNATURES = {
    "psi_status_str": (C.c_char_p, [_i]),
    "psi_create": (_i, [_P, _P, _P]),
    "psi_destroy": (_i, [_P]),
    "psi_set_stream": (_i, [_P, _P]),
    "psi_build": (_i, [_P, _P, _u64]),
    "psi_batch_insert": (_i, [_P, _P, _u64, _P]),
    "psi_batch_delete": (_i, [_P, _P, _u64, _P]),
    "psi_knn": (_i, [_P, _P, _u64, _u32, _P, _P]),
    "psi_range_count": (_i, [_P, _P, _u64, _P]),
    "psi_range_report": (_i, [_P, _P, _u64, _P, _P]),
    "psi_sync": (_i, [_P]),
    "psi_size": (_i, [_P, _P]),
    "psi_next_id": (_i, [_P, _P]),
    "psi_export": (_i, [_P, _P, _P, _P]),
    "psi_shape": (_i, [_P, _P, _P, _P]),
    "psi_export_structure": (_i, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "psi_export_leaves": (_i, [_P, _P, _P]),
    "psi_encode": (_i, [_u32, _u32, _P, _u64, _P, _P]),
    "psi_sort_pairs": (_i, [_P, _P, _u64, _P, _P, _P]),
    "psi_sort_pairs_noalloc": (_i, [_P, _P, _u64, _P, _P, _P]),
    "psi_multi_build": (_i, [_P, _P, _u32, _P, _P, _P]),
    "psi_multi_destroy": (_i, [_P]),
    "psi_multi_knn": (_i, [_P, _P, _P, _u32, _P, _P]),
    "psi_multi_sync": (_i, [_P]),
    "psi_multi_shape": (_i, [_P, _u32, _P, _P, _P]),
    "psi_multi_export_structure": (_i, [_P, _u32, _P, _P, _P, _P, _P, _P, _P, _P]),
    "psi_multi_export": (_i, [_P, _P, _P, _P]),
    "psi_server_create": (_i, [_P, _u64, _P]),
    "psi_server_destroy": (_i, [_P]),
    "psi_server_submit": (_i, [_P, _P, _P]),
    "psi_server_poll": (_i, [_P, _u64, _P, _P]),
    "psi_server_wait": (_i, [_P, _u64, _P]),
    "psi_server_flush": (_i, [_P]),
    "psi_graph_begin": (_i, [_P]),
    "psi_graph_end": (_i, [_P, _P]),
    "psi_graph_launch": (_i, [_P, _P]),
    "psi_graph_destroy": (_i, [_P]),
    "psi_orth_create": (_i, [_P, _P, _P]),
    "psi_orth_destroy": (_i, [_P]),
    "psi_orth_build": (_i, [_P, _P, _u64]),
    "psi_orth_batch_insert": (_i, [_P, _P, _u64, _P]),
    "psi_orth_batch_delete": (_i, [_P, _P, _u64, _P]),
    "psi_orth_size": (_i, [_P, _P, _P]),
    "psi_orth_knn": (_i, [_P, _P, _u64, _u32, _P, _P]),
    "psi_orth_range_count": (_i, [_P, _P, _u64, _P]),
    "psi_orth_range_report": (_i, [_P, _P, _u64, _P, _P]),
    "psi_orth_sync": (_i, [_P]),
    "psi_orth_shape": (_i, [_P, _P, _P, _P]),
    "psi_orth_export": (_i, [_P, _P, _P]),
    "psi_orth_prof_enable": (_i, [_P, _i]),
    "psi_orth_prof_reset": (_i, [_P]),
    "psi_orth_prof_get": (_i, [_P, C.c_char_p, _P, _P, _P]),
    "psi_prof_enable": (_i, [_P, _i]),
    "psi_query_stats": (_i, [_P, _i, _P]),
    "psi_bst_create": (_i, [_u32, _u32, _u32, _P, _P]),
    "psi_bst_destroy": (_i, [_P]),
    "psi_bst_build": (_i, [_P, _P, _u64]),
    "psi_bst_batch_insert": (_i, [_P, _P, _u64, _P]),
    "psi_bst_batch_delete": (_i, [_P, _P, _u64, _P]),
    "psi_bst_knn": (_i, [_P, _P, _u64, _u32, _P, _P]),
    "psi_bst_range_count": (_i, [_P, _P, _u64, _P]),
    "psi_bst_range_report": (_i, [_P, _P, _u64, _P, _P]),
    "psi_bst_sync": (_i, [_P]),
    "psi_bst_shape": (_i, [_P, _P, _P, _P, _P]),
    "psi_bst_export": (_i, [_P, _P, _P, _P, _P]),
    "psi_set_tuning": (_i, [_P, _P]),
    "psi_get_tuning": (_i, [_P, _P]),
    "psi_prof_only": (_i, [_P, C.c_char_p]),
    "psi_prof_reset": (_i, [_P]),
    "psi_prof_get": (_i, [_P, C.c_char_p, _P, _P, _P]),
}


class PsiError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {STATUS.get(code, code)}")
        self.code = code


class psi_params(C.Structure):
    _fields_ = [("dim", C.c_uint32), ("curve", C.c_uint32), ("leaf_size", C.c_uint32),
                ("fanout", C.c_uint32), ("flags", C.c_uint32)]


REQ_INSERT, REQ_DELETE, REQ_KNN, REQ_RANGE_COUNT, REQ_RANGE_REPORT = 0, 1, 2, 3, 4


class psi_request(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("k", C.c_uint32), ("n", C.c_uint64), ("d_in", C.c_void_p),
                ("d_ids", C.c_void_p), ("d_out", C.c_void_p), ("ids_cap", C.c_uint64),
                ("ready_event", C.c_void_p)]


_lib = None


def lib():
    """Load libpsi.so (built by paper_2601_05347_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_2601_05347_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int, where: str):
    if code != 0:
        raise PsiError(code, where)


def _torch():
    import torch
    return torch


def _dev_ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _as_u32(x, dev):
    """host array or tensor -> contiguous int32 device tensor holding u32 bits"""
    torch = _torch()
    if isinstance(x, torch.Tensor):
        if x.dtype not in (torch.int32, torch.uint32):
            raise ValueError("expected 32-bit integer tensor")
        t = x.to(dev).contiguous()
        return t.view(torch.int32) if t.dtype == torch.uint32 else t
    a = np.ascontiguousarray(x, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).to(dev)


def _as_u64(x, dev):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        t = x.to(dev).contiguous()
        return t.view(torch.int64) if t.dtype == torch.uint64 else t
    a = np.ascontiguousarray(x, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(dev)


def to_u32(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def to_u64(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


# ------------------------------------------------------------ C ABI mirrors

def psi_status_str(code: int) -> str:
    return lib().psi_status_str(code).decode()


def psi_create(dim: int, curve: int, leaf_size: int = 32, fanout: int = 8, flags: int = 0, stream=None):
    h = C.c_void_p()
    prm = psi_params(dim, curve, leaf_size, fanout, flags)
    _check(lib().psi_create(C.byref(prm), _stream_ptr(stream), C.byref(h)), "psi_create")
    return h


def psi_destroy(h):
    _check(lib().psi_destroy(h), "psi_destroy")


def psi_set_stream(h, stream=None):
    _check(lib().psi_set_stream(h, _stream_ptr(stream)), "psi_set_stream")


def psi_build(h, pts, n: int):
    _check(lib().psi_build(h, _dev_ptr(pts), n), "psi_build")


def psi_batch_insert(h, pts, m: int, new_ids=None):
    _check(lib().psi_batch_insert(h, _dev_ptr(pts), m, _dev_ptr(new_ids)), "psi_batch_insert")


def psi_batch_delete(h, ids, m: int, ndeleted=None):
    _check(lib().psi_batch_delete(h, _dev_ptr(ids), m, _dev_ptr(ndeleted)), "psi_batch_delete")


def psi_knn(h, q, nq: int, k: int, ids, d2):
    _check(lib().psi_knn(h, _dev_ptr(q), nq, k, _dev_ptr(ids), _dev_ptr(d2)), "psi_knn")


def psi_range_count(h, boxes, nb: int, counts):
    _check(lib().psi_range_count(h, _dev_ptr(boxes), nb, _dev_ptr(counts)), "psi_range_count")


def psi_range_report(h, boxes, nb: int, offsets, ids):
    _check(lib().psi_range_report(h, _dev_ptr(boxes), nb, _dev_ptr(offsets), _dev_ptr(ids)),
           "psi_range_report")


def psi_sync(h):
    _check(lib().psi_sync(h), "psi_sync")


def psi_size(h) -> int:
    v = C.c_uint64()
    _check(lib().psi_size(h, C.byref(v)), "psi_size")
    return v.value


def psi_next_id(h) -> int:
    v = C.c_uint32()
    _check(lib().psi_next_id(h, C.byref(v)), "psi_next_id")
    return v.value


def psi_export(h, keys, ids, pts):
    _check(lib().psi_export(h, _dev_ptr(keys), _dev_ptr(ids), _dev_ptr(pts)), "psi_export")


def psi_shape(h):
    L = C.c_uint64()
    hh = C.c_uint32()
    sizes = (C.c_uint64 * 64)()
    _check(lib().psi_shape(h, C.byref(L), C.byref(hh), sizes), "psi_shape")
    return L.value, hh.value, [sizes[i] for i in range(hh.value + 1)] if L.value else []


def psi_export_structure(h, piv_key, piv_id, leaf_cnt, leaf_lo, leaf_hi, node_lo, node_hi, node_cnt):
    _check(lib().psi_export_structure(h, *[_dev_ptr(t) for t in (piv_key, piv_id, leaf_cnt, leaf_lo, leaf_hi,
                                                                  node_lo, node_hi, node_cnt)]),
           "psi_export_structure")


def psi_export_leaves(h, ids, pts):
    _check(lib().psi_export_leaves(h, _dev_ptr(ids), _dev_ptr(pts)), "psi_export_leaves")


def psi_encode(dim: int, curve: int, pts, n: int, keys, stream=None):
    _check(lib().psi_encode(dim, curve, _dev_ptr(pts), n, _dev_ptr(keys), _stream_ptr(stream)), "psi_encode")


def psi_sort_pairs(keys, ids, n: int, keys_out, ids_out, stream=None):
    _check(lib().psi_sort_pairs(_dev_ptr(keys), _dev_ptr(ids), n, _dev_ptr(keys_out), _dev_ptr(ids_out),
                                _stream_ptr(stream)), "psi_sort_pairs")


SORT_NOALLOC_MAX = 1 << 20


def psi_sort_pairs_noalloc(keys, ids, n: int, keys_out, ids_out, stream=None):
    _check(lib().psi_sort_pairs_noalloc(_dev_ptr(keys), _dev_ptr(ids), n, _dev_ptr(keys_out), _dev_ptr(ids_out),
                                        _stream_ptr(stream)), "psi_sort_pairs_noalloc")


def psi_multi_build(dim: int, curve: int, num: int, pt_off, pts, leaf_size: int = 32, fanout: int = 8,
                    stream=None):
    h = C.c_void_p()
    prm = psi_params(dim, curve, leaf_size, fanout, 0)
    _check(lib().psi_multi_build(C.byref(prm), _stream_ptr(stream), num, _dev_ptr(pt_off), _dev_ptr(pts),
                                 C.byref(h)), "psi_multi_build")
    return h


def psi_multi_destroy(h):
    _check(lib().psi_multi_destroy(h), "psi_multi_destroy")


def psi_multi_knn(h, q_off, q, k: int, ids, d2):
    _check(lib().psi_multi_knn(h, _dev_ptr(q_off), _dev_ptr(q), k, _dev_ptr(ids), _dev_ptr(d2)), "psi_multi_knn")


def psi_multi_sync(h):
    _check(lib().psi_multi_sync(h), "psi_multi_sync")


def psi_multi_shape(h, index: int):
    L = C.c_uint64()
    hh = C.c_uint32()
    sizes = (C.c_uint64 * 64)()
    _check(lib().psi_multi_shape(h, index, C.byref(L), C.byref(hh), sizes), "psi_multi_shape")
    return L.value, hh.value, [sizes[i] for i in range(hh.value + 1)] if L.value else []


def psi_multi_export_structure(h, index, piv_key, piv_id, leaf_cnt, leaf_lo, leaf_hi, node_lo, node_hi, node_cnt):
    _check(lib().psi_multi_export_structure(h, index, *[_dev_ptr(t) for t in (piv_key, piv_id, leaf_cnt, leaf_lo,
                                                                              leaf_hi, node_lo, node_hi, node_cnt)]),
           "psi_multi_export_structure")


def psi_multi_export(h, keys, ids, pts):
    _check(lib().psi_multi_export(h, _dev_ptr(keys), _dev_ptr(ids), _dev_ptr(pts)), "psi_multi_export")


def psi_server_create(h, budget_bytes: int):
    s = C.c_void_p()
    _check(lib().psi_server_create(h, budget_bytes, C.byref(s)), "psi_server_create")
    return s


def psi_server_destroy(s):
    _check(lib().psi_server_destroy(s), "psi_server_destroy")


def psi_server_submit(s, kind: int, n: int, d_in, d_ids=None, d_out=None, k: int = 0, ids_cap: int = 0,
                      ready_event=None) -> int:
    r = psi_request(kind, k, n, _dev_ptr(d_in), _dev_ptr(d_ids), _dev_ptr(d_out), ids_cap,
                    C.c_void_p(ready_event.cuda_event) if ready_event is not None else None)
    t = C.c_uint64()
    _check(lib().psi_server_submit(s, C.byref(r), C.byref(t)), "psi_server_submit")
    return t.value


def psi_server_poll(s, ticket: int):
    """(done, completion ms since the server was created or None)."""
    d = C.c_int()
    ms = C.c_double(-1.0)
    _check(lib().psi_server_poll(s, ticket, C.byref(d), C.byref(ms)), "psi_server_poll")
    return bool(d.value), (ms.value if d.value else None)


def psi_server_wait(s, ticket: int) -> float:
    ms = C.c_double(-1.0)
    _check(lib().psi_server_wait(s, ticket, C.byref(ms)), "psi_server_wait")
    return ms.value


def psi_server_flush(s):
    _check(lib().psi_server_flush(s), "psi_server_flush")


def psi_graph_begin(stream=None):
    _check(lib().psi_graph_begin(_stream_ptr(stream)), "psi_graph_begin")


def psi_graph_end(stream=None):
    g = C.c_void_p()
    _check(lib().psi_graph_end(_stream_ptr(stream), C.byref(g)), "psi_graph_end")
    return g


def psi_graph_launch(g, stream=None):
    _check(lib().psi_graph_launch(g, _stream_ptr(stream)), "psi_graph_launch")


def psi_graph_destroy(g):
    _check(lib().psi_graph_destroy(g), "psi_graph_destroy")


class psi_tuning(C.Structure):
    _fields_ = [("knn_seed_leaves", C.c_uint32), ("knn_cand", C.c_uint32), ("order_bits", C.c_uint32)]


def psi_set_tuning(h, knn_seed_leaves: int = 3, knn_cand: int = 16, order_bits: int = 24):
    t = psi_tuning(knn_seed_leaves, knn_cand, order_bits)
    _check(lib().psi_set_tuning(h, C.byref(t)), "psi_set_tuning")


def psi_get_tuning(h) -> dict:
    t = psi_tuning()
    _check(lib().psi_get_tuning(h, C.byref(t)), "psi_get_tuning")
    return {"knn_seed_leaves": t.knn_seed_leaves, "knn_cand": t.knn_cand, "order_bits": t.order_bits}


def psi_query_stats(h, enable: bool):
    """kNN walk counts so far [queries, box tests, leaves, points] (numpy
    u64), then counting switched on or off."""
    out = np.zeros(4, np.uint64)
    _check(lib().psi_query_stats(h, 1 if enable else 0, out.ctypes.data),
           "psi_query_stats")
    return out


def psi_prof_enable(h, on: bool):
    _check(lib().psi_prof_enable(h, 1 if on else 0), "psi_prof_enable")


def psi_prof_only(h, family):
    _check(lib().psi_prof_only(h, family.encode() if family else None), "psi_prof_only")


def psi_prof_reset(h):
    _check(lib().psi_prof_reset(h), "psi_prof_reset")


def psi_prof_get(h, family: str):
    ms = C.c_double()
    n = C.c_uint64()
    b = C.c_uint64()
    _check(lib().psi_prof_get(h, family.encode(), C.byref(ms), C.byref(n), C.byref(b)), "psi_prof_get")
    return ms.value, n.value, b.value


def psi_orth_create(dim: int, leaf_size: int = 32, flags: int = 0, stream=None):
    h = C.c_void_p()
    prm = psi_params(dim, MORTON, leaf_size, 8, flags)
    _check(lib().psi_orth_create(C.byref(prm), _stream_ptr(stream), C.byref(h)), "psi_orth_create")
    return h


def psi_orth_destroy(h):
    _check(lib().psi_orth_destroy(h), "psi_orth_destroy")


def psi_orth_build(h, pts, n: int):
    _check(lib().psi_orth_build(h, _dev_ptr(pts), n), "psi_orth_build")


def psi_orth_batch_insert(h, pts, m: int, new_ids=None):
    _check(lib().psi_orth_batch_insert(h, _dev_ptr(pts), m, _dev_ptr(new_ids)), "psi_orth_batch_insert")


def psi_orth_batch_delete(h, ids, m: int, ndeleted=None):
    _check(lib().psi_orth_batch_delete(h, _dev_ptr(ids), m, _dev_ptr(ndeleted)), "psi_orth_batch_delete")


def psi_orth_size(h):
    n = C.c_uint64()
    nid = C.c_uint32()
    _check(lib().psi_orth_size(h, C.byref(n), C.byref(nid)), "psi_orth_size")
    return n.value, nid.value


def psi_orth_knn(h, q, nq: int, k: int, ids, d2):
    _check(lib().psi_orth_knn(h, _dev_ptr(q), nq, k, _dev_ptr(ids), _dev_ptr(d2)), "psi_orth_knn")


def psi_orth_range_count(h, boxes, nb: int, counts):
    _check(lib().psi_orth_range_count(h, _dev_ptr(boxes), nb, _dev_ptr(counts)), "psi_orth_range_count")


def psi_orth_range_report(h, boxes, nb: int, offsets, ids):
    _check(lib().psi_orth_range_report(h, _dev_ptr(boxes), nb, _dev_ptr(offsets), _dev_ptr(ids)),
           "psi_orth_range_report")


def psi_orth_sync(h):
    _check(lib().psi_orth_sync(h), "psi_orth_sync")


def psi_orth_shape(h):
    nn = C.c_uint64()
    nl = C.c_uint64()
    hh = C.c_uint32()
    _check(lib().psi_orth_shape(h, C.byref(nn), C.byref(nl), C.byref(hh)), "psi_orth_shape")
    return nn.value, nl.value, hh.value


def psi_orth_export(h, nodes, pts):
    _check(lib().psi_orth_export(h, _dev_ptr(nodes), _dev_ptr(pts)), "psi_orth_export")


def psi_orth_prof_enable(h, on: bool):
    _check(lib().psi_orth_prof_enable(h, 1 if on else 0), "psi_orth_prof_enable")


def psi_orth_prof_reset(h):
    _check(lib().psi_orth_prof_reset(h), "psi_orth_prof_reset")


def psi_orth_prof_get(h, family: str):
    ms = C.c_double()
    n = C.c_uint64()
    b = C.c_uint64()
    _check(lib().psi_orth_prof_get(h, family.encode(), C.byref(ms), C.byref(n), C.byref(b)), "psi_orth_prof_get")
    return ms.value, n.value, b.value


# ------------------------------------------------------------ convenience

class Index:
    """A SPaC-tree on the current ROCm device, bound to one stream."""

    def __init__(self, dim: int, curve: int, leaf_size: int = 32, fanout: int = 8, device="cuda", stream=None,
                 flags: int = 0):
        torch = _torch()
        self.dim, self.curve, self.leaf_size, self.fanout = dim, curve, leaf_size, fanout
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = psi_create(dim, curve, leaf_size, fanout, flags, self.stream)

    def close(self):
        if getattr(self, "_h", None):
            psi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _pts(self, pts):
        t = _as_u32(pts, self.device)
        return t.reshape(-1, self.dim).contiguous()

    def build(self, pts):
        t = self._pts(pts)
        psi_build(self._h, t, t.shape[0])
        return self

    def batch_insert(self, pts):
        torch = _torch()
        t = self._pts(pts)
        ids = torch.empty(t.shape[0], dtype=torch.int32, device=self.device)
        psi_batch_insert(self._h, t, t.shape[0], ids)
        return ids

    def batch_delete(self, ids) -> int:
        torch = _torch()
        t = _as_u32(ids, self.device).reshape(-1)
        nd = torch.zeros(1, dtype=torch.int64, device=self.device)
        psi_batch_delete(self._h, t, t.numel(), nd)
        return nd

    def knn(self, q, k: int):
        torch = _torch()
        t = self._pts(q)
        nq = t.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int32, device=self.device)
        d2 = torch.empty((nq, k), dtype=torch.int64, device=self.device)
        psi_knn(self._h, t, nq, k, ids, d2)
        return ids, d2

    def range_count(self, boxes):
        torch = _torch()
        b = _as_u32(boxes, self.device).reshape(-1, 2, self.dim).contiguous()
        cnt = torch.empty(b.shape[0], dtype=torch.int64, device=self.device)
        psi_range_count(self._h, b, b.shape[0], cnt)
        return cnt

    def range_report(self, boxes, counts=None):
        """Returns (offsets[nb+1], ids). Counts are computed if not given."""
        torch = _torch()
        b = _as_u32(boxes, self.device).reshape(-1, 2, self.dim).contiguous()
        cnt = self.range_count(b) if counts is None else counts
        off = torch.zeros(b.shape[0] + 1, dtype=torch.int64, device=self.device)
        torch.cumsum(cnt, 0, out=off[1:])
        total = int(off[-1].item())
        ids = torch.empty(max(total, 1), dtype=torch.int32, device=self.device)
        psi_range_report(self._h, b, b.shape[0], off, ids)
        return off, ids[:total]

    def sync(self):
        psi_sync(self._h)

    def size(self) -> int:
        return psi_size(self._h)

    def next_id(self) -> int:
        return psi_next_id(self._h)

    def export(self):
        """Live entries in (key, id) order as numpy (keys u64, ids u32, pts u32[n, dim])."""
        torch = _torch()
        n = self.size()
        k = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        i = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        p = torch.empty((max(n, 1), self.dim), dtype=torch.int32, device=self.device)
        psi_export(self._h, k, i, p)
        self.sync()
        return to_u64(k[:n]), to_u32(i[:n]), to_u32(p[:n])

    def shape(self):
        return psi_shape(self._h)

    def structure(self) -> dict:
        torch = _torch()
        L, h, sizes = self.shape()
        nn = int(sum(sizes)) if L else 0
        D, dev = self.dim, self.device
        t = dict(piv_key=torch.empty(max(L, 1), dtype=torch.int64, device=dev),
                 piv_id=torch.empty(max(L, 1), dtype=torch.int32, device=dev),
                 leaf_cnt=torch.empty(max(L, 1), dtype=torch.int32, device=dev),
                 leaf_lo=torch.empty((max(L, 1), D), dtype=torch.int32, device=dev),
                 leaf_hi=torch.empty((max(L, 1), D), dtype=torch.int32, device=dev),
                 node_lo=torch.empty((max(nn, 1), D), dtype=torch.int32, device=dev),
                 node_hi=torch.empty((max(nn, 1), D), dtype=torch.int32, device=dev),
                 node_cnt=torch.empty(max(nn, 1), dtype=torch.int64, device=dev))
        psi_export_structure(self._h, t["piv_key"], t["piv_id"], t["leaf_cnt"], t["leaf_lo"], t["leaf_hi"],
                             t["node_lo"], t["node_hi"], t["node_cnt"])
        self.sync()
        out = dict(n_leaves=L, height=h, level_sizes=np.array(sizes, dtype=np.int64))
        for name, ten in t.items():
            cut = ten[:L] if name.startswith(("piv", "leaf")) else ten[:nn]
            out[name] = to_u64(cut) if ten.dtype == torch.int64 else to_u32(cut)
        return out

    def leaves(self):
        """Raw leaf contents (stored order) and per-leaf counts."""
        torch = _torch()
        n = self.size()
        i = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        p = torch.empty((max(n, 1), self.dim), dtype=torch.int32, device=self.device)
        psi_export_leaves(self._h, i, p)
        self.sync()
        return to_u32(i[:n]), to_u32(p[:n])

    # timing
    def prof_enable(self, on=True):
        psi_prof_enable(self._h, on)

    def prof_only(self, family=None):
        psi_prof_only(self._h, family)

    def prof_reset(self):
        psi_prof_reset(self._h)

    def prof_get(self, family: str):
        return psi_prof_get(self._h, family)


ORTH_LEAF = 0x80000000


class Orth:
    """A P-Orth tree (quadtree / octree) on the current ROCm device."""

    def __init__(self, dim: int, leaf_size: int = 32, device="cuda", stream=None, flags: int = 0):
        torch = _torch()
        self.dim, self.leaf_size = dim, leaf_size
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = psi_orth_create(dim, leaf_size, flags, self.stream)
        self.n = 0

    def close(self):
        if getattr(self, "_h", None):
            psi_orth_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _pts(self, pts):
        return _as_u32(pts, self.device).reshape(-1, self.dim).contiguous()

    def build(self, pts):
        t = self._pts(pts)
        try:
            psi_orth_build(self._h, t, t.shape[0])
        finally:
            self.n = psi_orth_size(self._h)[0]
        return self

    def batch_insert(self, pts):
        torch = _torch()
        t = self._pts(pts)
        ids = torch.empty(max(t.shape[0], 1), dtype=torch.int32, device=self.device)
        try:
            psi_orth_batch_insert(self._h, t, t.shape[0], ids)
        finally:
            self.n = psi_orth_size(self._h)[0]
        return ids[:t.shape[0]]

    def batch_delete(self, ids) -> int:
        torch = _torch()
        t = _as_u32(ids, self.device).reshape(-1)
        nd = torch.zeros(1, dtype=torch.int64, device=self.device)
        try:
            psi_orth_batch_delete(self._h, t, t.numel(), nd)
        finally:
            self.n = psi_orth_size(self._h)[0]
        return int(nd.item())

    def size(self):
        """(live points, next id)"""
        return psi_orth_size(self._h)

    def knn(self, q, k: int):
        torch = _torch()
        t = self._pts(q)
        nq = t.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int32, device=self.device)
        d2 = torch.empty((nq, k), dtype=torch.int64, device=self.device)
        psi_orth_knn(self._h, t, nq, k, ids, d2)
        return ids, d2

    def range_count(self, boxes):
        torch = _torch()
        b = _as_u32(boxes, self.device).reshape(-1, 2, self.dim).contiguous()
        cnt = torch.empty(b.shape[0], dtype=torch.int64, device=self.device)
        psi_orth_range_count(self._h, b, b.shape[0], cnt)
        return cnt

    def range_report(self, boxes, counts=None):
        """Returns (offsets[nb+1], ids); ids of a box in the tree's preorder."""
        torch = _torch()
        b = _as_u32(boxes, self.device).reshape(-1, 2, self.dim).contiguous()
        cnt = self.range_count(b) if counts is None else counts
        off = torch.zeros(b.shape[0] + 1, dtype=torch.int64, device=self.device)
        torch.cumsum(cnt, 0, out=off[1:])
        total = int(off[-1].item())
        ids = torch.empty(max(total, 1), dtype=torch.int32, device=self.device)
        psi_orth_range_report(self._h, b, b.shape[0], off, ids)
        return off, ids[:total]

    def sync(self):
        psi_orth_sync(self._h)

    def shape(self):
        """(nodes, leaves, height)"""
        return psi_orth_shape(self._h)

    def export(self):
        """(nodes u32[N, 8], pts u32[n, 4]) as numpy; layout in include/psi.h."""
        torch = _torch()
        N = self.shape()[0]
        nodes = torch.empty((max(N, 1), 8), dtype=torch.int32, device=self.device)
        pts = torch.empty((max(self.n, 1), 4), dtype=torch.int32, device=self.device)
        psi_orth_export(self._h, nodes, pts)
        return to_u32(nodes[:N]), to_u32(pts[:self.n])

    def prof_enable(self, on=True):
        psi_orth_prof_enable(self._h, on)

    def prof_reset(self):
        psi_orth_prof_reset(self._h)

    def prof_get(self, family: str):
        return psi_orth_prof_get(self._h, family)


def psi_bst_create(dim: int, curve: int, leaf_wrap: int, stream=None):
    h = C.c_void_p()
    _check(lib().psi_bst_create(dim, curve, leaf_wrap, _stream_ptr(stream) if stream is not None else None,
                                C.byref(h)), "psi_bst_create")
    return h


def psi_bst_destroy(h):
    _check(lib().psi_bst_destroy(h), "psi_bst_destroy")


def psi_bst_sync(h):
    _check(lib().psi_bst_sync(h), "psi_bst_sync")


def psi_bst_shape(h):
    n, root, ns, ls = C.c_uint64(), C.c_uint32(), C.c_uint64(), C.c_uint64()
    _check(lib().psi_bst_shape(h, C.byref(n), C.byref(root), C.byref(ns), C.byref(ls)), "psi_bst_shape")
    return n.value, root.value, ns.value, ls.value


def psi_bst_export(h, nodes, leaves, ids, pts):
    _check(lib().psi_bst_export(h, _dev_ptr(nodes), _dev_ptr(leaves), _dev_ptr(ids), _dev_ptr(pts)), "psi_bst_export")


def psi_bst_build(h, pts, n: int):
    _check(lib().psi_bst_build(h, _dev_ptr(pts), n), "psi_bst_build")


def psi_bst_batch_insert(h, pts, m: int, new_ids):
    _check(lib().psi_bst_batch_insert(h, _dev_ptr(pts), m, _dev_ptr(new_ids)), "psi_bst_batch_insert")


def psi_bst_batch_delete(h, ids, m: int, ndeleted=None):
    _check(lib().psi_bst_batch_delete(h, _dev_ptr(ids), m, _dev_ptr(ndeleted)), "psi_bst_batch_delete")


def psi_bst_knn(h, q, nq: int, k: int, ids, d2):
    _check(lib().psi_bst_knn(h, _dev_ptr(q), nq, k, _dev_ptr(ids), _dev_ptr(d2)), "psi_bst_knn")


def psi_bst_range_count(h, boxes, nb: int, counts):
    _check(lib().psi_bst_range_count(h, _dev_ptr(boxes), nb, _dev_ptr(counts)), "psi_bst_range_count")


def psi_bst_range_report(h, boxes, nb: int, offsets, ids):
    _check(lib().psi_bst_range_report(h, _dev_ptr(boxes), nb, _dev_ptr(offsets), _dev_ptr(ids)),
           "psi_bst_range_report")


class Bst:
    """The SPaC-tree in the paper's own shape (BuildSorted, Sec. 4) on the
    current ROCm device, bound to one stream."""

    def __init__(self, dim: int, curve: int, leaf_wrap: int = 40, device="cuda", stream=None):
        torch = _torch()
        self.dim, self.curve, self.leaf_wrap = dim, curve, leaf_wrap
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().psi_bst_create(dim, curve, leaf_wrap, _stream_ptr(self.stream), C.byref(h)), "psi_bst_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().psi_bst_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _pts(self, pts):
        return _as_u32(pts, self.device).reshape(-1, self.dim).contiguous()

    def build(self, pts):
        t = self._pts(pts)
        _check(lib().psi_bst_build(self._h, _dev_ptr(t), t.shape[0]), "psi_bst_build")
        return self

    def batch_insert(self, pts):
        torch = _torch()
        t = self._pts(pts)
        ids = torch.empty(max(t.shape[0], 1), dtype=torch.int32, device=self.device)
        _check(lib().psi_bst_batch_insert(self._h, _dev_ptr(t), t.shape[0], _dev_ptr(ids)), "psi_bst_batch_insert")
        return ids[:t.shape[0]]

    def batch_delete(self, ids):
        torch = _torch()
        t = _as_u32(ids, self.device).reshape(-1)
        nd = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(lib().psi_bst_batch_delete(self._h, _dev_ptr(t), t.numel(), _dev_ptr(nd)), "psi_bst_batch_delete")
        return nd

    def knn(self, q, k: int):
        torch = _torch()
        t = self._pts(q)
        nq = t.shape[0]
        ids = torch.empty((max(nq, 1), k), dtype=torch.int32, device=self.device)
        d2 = torch.empty((max(nq, 1), k), dtype=torch.int64, device=self.device)
        _check(lib().psi_bst_knn(self._h, _dev_ptr(t), nq, k, _dev_ptr(ids), _dev_ptr(d2)), "psi_bst_knn")
        return ids[:nq], d2[:nq]

    def range_count(self, boxes):
        torch = _torch()
        b = _as_u32(boxes, self.device).reshape(-1, 2, self.dim).contiguous()
        cnt = torch.empty(max(b.shape[0], 1), dtype=torch.int64, device=self.device)
        _check(lib().psi_bst_range_count(self._h, _dev_ptr(b), b.shape[0], _dev_ptr(cnt)), "psi_bst_range_count")
        return cnt[:b.shape[0]]

    def range_report(self, boxes, counts=None):
        torch = _torch()
        b = _as_u32(boxes, self.device).reshape(-1, 2, self.dim).contiguous()
        cnt = self.range_count(b) if counts is None else counts
        off = torch.zeros(b.shape[0] + 1, dtype=torch.int64, device=self.device)
        torch.cumsum(cnt, 0, out=off[1:])
        total = int(off[-1].item())
        ids = torch.empty(max(total, 1), dtype=torch.int32, device=self.device)
        _check(lib().psi_bst_range_report(self._h, _dev_ptr(b), b.shape[0], _dev_ptr(off), _dev_ptr(ids)),
               "psi_bst_range_report")
        return off, ids[:total]

    def sync(self):
        _check(lib().psi_bst_sync(self._h), "psi_bst_sync")

    def shape(self):
        """(points, root reference, node slots, leaf slots)."""
        return psi_bst_shape(self._h)

    def export(self) -> dict:
        """The pools as numpy arrays: node records (16 words), leaf records
        (8 words), each leaf slot's ids and points, and the root."""
        torch = _torch()
        n, root, ns, ls = self.shape()
        w = self.leaf_wrap
        nodes = torch.empty(max(ns, 1) * 16, dtype=torch.int32, device=self.device)
        leaves = torch.empty(max(ls, 1) * 8, dtype=torch.int32, device=self.device)
        ids = torch.empty(max(ls, 1) * w, dtype=torch.int32, device=self.device)
        pts = torch.empty(max(ls, 1) * w * self.dim, dtype=torch.int32, device=self.device)
        psi_bst_export(self._h, nodes, leaves, ids, pts)
        return {"n": n, "root": root, "nodes": to_u32(nodes)[:ns * 16].reshape(ns, 16),
                "leaves": to_u32(leaves)[:ls * 8].reshape(ls, 8), "ids": to_u32(ids)[:ls * w].reshape(ls, w),
                "pts": to_u32(pts)[:ls * w * self.dim].reshape(ls, w, self.dim), "leaf_wrap": w}


class MultiIndex:
    """Many independent SPaC-trees built and queried together (one CSR batch)."""

    def __init__(self, dim: int, curve: int, pt_off, pts, leaf_size: int = 32, fanout: int = 8, device="cuda"):
        torch = _torch()
        self.dim, self.curve = dim, curve
        self.device = torch.device(device)
        self.off = _as_u64(pt_off, self.device).reshape(-1).contiguous()
        self.num = self.off.numel() - 1
        p = _as_u32(pts, self.device).reshape(-1, dim).contiguous()
        self._h = psi_multi_build(dim, curve, self.num, self.off, p, leaf_size, fanout)
        self.n_total = p.shape[0]

    def close(self):
        if getattr(self, "_h", None):
            psi_multi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def knn(self, q_off, q, k: int):
        torch = _torch()
        qo = _as_u64(q_off, self.device).reshape(-1).contiguous()
        qq = _as_u32(q, self.device).reshape(-1, self.dim).contiguous()
        nq = qq.shape[0]
        ids = torch.empty((max(nq, 1), k), dtype=torch.int32, device=self.device)
        d2 = torch.empty((max(nq, 1), k), dtype=torch.int64, device=self.device)
        psi_multi_knn(self._h, qo, qq, k, ids, d2)
        return ids[:nq], d2[:nq]

    def sync(self):
        psi_multi_sync(self._h)

    def export(self):
        torch = _torch()
        n = self.n_total
        k = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        i = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        p = torch.empty((max(n, 1), self.dim), dtype=torch.int32, device=self.device)
        psi_multi_export(self._h, k, i, p)
        self.sync()
        return to_u64(k[:n]), to_u32(i[:n]), to_u32(p[:n])

    def structure(self, index: int) -> dict:
        torch = _torch()
        L, h, sizes = psi_multi_shape(self._h, index)
        nn = int(sum(sizes)) if L else 0
        D, dev = self.dim, self.device
        t = dict(piv_key=torch.empty(max(L, 1), dtype=torch.int64, device=dev),
                 piv_id=torch.empty(max(L, 1), dtype=torch.int32, device=dev),
                 leaf_cnt=torch.empty(max(L, 1), dtype=torch.int32, device=dev),
                 leaf_lo=torch.empty((max(L, 1), D), dtype=torch.int32, device=dev),
                 leaf_hi=torch.empty((max(L, 1), D), dtype=torch.int32, device=dev),
                 node_lo=torch.empty((max(nn, 1), D), dtype=torch.int32, device=dev),
                 node_hi=torch.empty((max(nn, 1), D), dtype=torch.int32, device=dev),
                 node_cnt=torch.empty(max(nn, 1), dtype=torch.int64, device=dev))
        psi_multi_export_structure(self._h, index, t["piv_key"], t["piv_id"], t["leaf_cnt"], t["leaf_lo"],
                                   t["leaf_hi"], t["node_lo"], t["node_hi"], t["node_cnt"])
        self.sync()
        out = dict(n_leaves=L, height=h, level_sizes=np.array(sizes, dtype=np.int64))
        for name, ten in t.items():
            cut = ten[:L] if name.startswith(("piv", "leaf")) else ten[:nn]
            out[name] = to_u64(cut) if ten.dtype == torch.int64 else to_u32(cut)
        return out


def encode(pts, dim: int, curve: int):
    """Curve keys of points on the GPU (returns an int64 tensor of u64 bits)."""
    torch = _torch()
    t = _as_u32(pts, "cuda").reshape(-1, dim).contiguous()
    keys = torch.empty(t.shape[0], dtype=torch.int64, device=t.device)
    psi_encode(dim, curve, t, t.shape[0], keys)
    return keys


def sort_pairs(keys, ids):
    """Stable sort of (key, id) pairs on the GPU; returns (keys, ids) tensors."""
    torch = _torch()
    k = _as_u64(keys, "cuda").reshape(-1)
    i = _as_u32(ids, "cuda").reshape(-1)
    ko = torch.empty_like(k)
    io = torch.empty_like(i)
    psi_sort_pairs(k, i, k.numel(), ko, io)
    return ko, io
