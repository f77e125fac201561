"""ctypes wrapper of the CPU oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users. The product path never imports this.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

MORTON, HILBERT = 0, 1
PAD_ID = 0xFFFFFFFF
PAD_D2 = 0xFFFFFFFFFFFFFFFF


def build_lib(force: bool = True) -> str:
    """Compile oracle.cpp with g++ into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("PSI_ORACLE_LIB")  # a test's planted-mistake copy
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build_lib(force=True)
        L = C.CDLL(path)
        P = C.c_void_p
        u64, u32, i32 = C.c_uint64, C.c_uint32, C.c_int
        sig = {
            "ora_morton": (u64, [i32, P]),
            "ora_hilbert": (u64, [i32, P]),
            "ora_encode": (None, [i32, i32, P, u64, P]),
            "ora_sort_pairs": (None, [u64, P, P]),
            "ora_new": (P, [i32, i32, u32, u32]),
            "ora_free": (None, [P]),
            "ora_build": (i32, [P, P, u64]),
            "ora_insert": (i32, [P, P, u64, P]),
            "ora_delete": (u64, [P, P, u64]),
            "ora_size": (u64, [P]),
            "ora_next_id": (u32, [P]),
            "ora_dump": (None, [P, P, P, P]),
            "ora_struct_shape": (None, [P, P, P, P]),
            "ora_struct": (None, [P, P, P, P, P, P, P, P, P]),
            "ora_knn": (None, [P, P, u64, u32, P, P, i32]),
            "ora_knn_fullsort": (None, [P, P, u64, u32, P, P]),
            "ora_range_count": (None, [P, P, u64, P, i32]),
            "ora_range_report": (None, [P, P, u64, P, P, i32]),
            "ora_knn_points": (None, [i32, P, u64, P, u64, u32, P, P, i32]),
            "ora_range_count_points": (None, [i32, P, u64, P, u64, P, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def morton(dim: int, p) -> int:
    a = _c(p, np.uint32)
    return int(lib().ora_morton(dim, _p(a)))


def hilbert(dim: int, p) -> int:
    a = _c(p, np.uint32)
    return int(lib().ora_hilbert(dim, _p(a)))


def encode(pts, dim: int, curve: int) -> np.ndarray:
    a = _c(pts, np.uint32).reshape(-1, dim)
    out = np.empty(a.shape[0], dtype=np.uint64)
    lib().ora_encode(dim, curve, _p(a), a.shape[0], _p(out))
    return out


def sort_pairs(keys, ids):
    k = _c(keys, np.uint64).copy()
    i = _c(ids, np.uint32).copy()
    lib().ora_sort_pairs(k.size, _p(k), _p(i))
    return k, i


def knn_points(pts, q, k: int, threads: int = 0):
    """Brute-force kNN over raw points (ids = row numbers)."""
    p = _c(pts, np.uint32)
    dim = p.shape[1]
    qq = _c(q, np.uint32).reshape(-1, dim)
    ids = np.empty((qq.shape[0], k), dtype=np.uint32)
    d2 = np.empty((qq.shape[0], k), dtype=np.uint64)
    lib().ora_knn_points(dim, _p(p), p.shape[0], _p(qq), qq.shape[0], k, _p(ids), _p(d2), threads)
    return ids, d2


def range_count_points(pts, boxes, threads: int = 0):
    p = _c(pts, np.uint32)
    dim = p.shape[1]
    b = _c(boxes, np.uint32).reshape(-1, 2, dim)
    out = np.empty(b.shape[0], dtype=np.uint64)
    lib().ora_range_count_points(dim, _p(p), p.shape[0], _p(b), b.shape[0], _p(out), threads)
    return out


class RefIndex:
    """The oracle's index: a sorted set of (key, id, point) entries."""

    def __init__(self, dim: int, curve: int, leaf_size: int = 32, fanout: int = 8):
        self.dim, self.curve, self.leaf_size, self.fanout = dim, curve, leaf_size, fanout
        self._h = lib().ora_new(dim, curve, leaf_size, fanout)
        if not self._h:
            raise ValueError("bad oracle parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.ora_free(h)
            self._h = None

    def build(self, pts):
        a = _c(pts, np.uint32).reshape(-1, self.dim)
        if lib().ora_build(self._h, _p(a), a.shape[0]) != 0:
            raise ValueError("coordinate out of range")

    def batch_insert(self, pts) -> np.ndarray:
        a = _c(pts, np.uint32).reshape(-1, self.dim)
        ids = np.empty(a.shape[0], dtype=np.uint32)
        rc = lib().ora_insert(self._h, _p(a), a.shape[0], _p(ids))
        if rc != 0:
            raise ValueError("coordinate out of range" if rc == -1 else "id space exhausted")
        return ids

    def batch_delete(self, ids) -> int:
        a = _c(ids, np.uint32)
        return int(lib().ora_delete(self._h, _p(a), a.size))

    def size(self) -> int:
        return int(lib().ora_size(self._h))

    def next_id(self) -> int:
        return int(lib().ora_next_id(self._h))

    def dump(self):
        n = self.size()
        k = np.empty(n, dtype=np.uint64)
        i = np.empty(n, dtype=np.uint32)
        p = np.empty((n, self.dim), dtype=np.uint32)
        lib().ora_dump(self._h, _p(k), _p(i), _p(p))
        return k, i, p

    def structure(self) -> dict:
        """Canonical structure of a fresh build of the current set."""
        L = C.c_uint64(0)
        h = C.c_uint32(0)
        sizes = np.zeros(64, dtype=np.uint64)
        lib().ora_struct_shape(self._h, C.byref(L), C.byref(h), _p(sizes))
        L, h = L.value, h.value
        D = self.dim
        nl = int(sizes[: h + 1].sum()) if L else 0
        out = dict(n_leaves=L, height=h, level_sizes=sizes[: h + 1].astype(np.int64) if L else np.zeros(0, np.int64),
                   piv_key=np.empty(L, np.uint64), piv_id=np.empty(L, np.uint32),
                   leaf_cnt=np.empty(L, np.uint32), leaf_lo=np.empty((L, D), np.uint32),
                   leaf_hi=np.empty((L, D), np.uint32), node_lo=np.empty((nl, D), np.uint32),
                   node_hi=np.empty((nl, D), np.uint32), node_cnt=np.empty(nl, np.uint64))
        if L:
            lib().ora_struct(self._h, _p(out["piv_key"]), _p(out["piv_id"]), _p(out["leaf_cnt"]),
                             _p(out["leaf_lo"]), _p(out["leaf_hi"]), _p(out["node_lo"]),
                             _p(out["node_hi"]), _p(out["node_cnt"]))
        return out

    def knn(self, q, k: int, threads: int = 0):
        a = _c(q, np.uint32).reshape(-1, self.dim)
        ids = np.empty((a.shape[0], k), dtype=np.uint32)
        d2 = np.empty((a.shape[0], k), dtype=np.uint64)
        lib().ora_knn(self._h, _p(a), a.shape[0], k, _p(ids), _p(d2), threads)
        return ids, d2

    def knn_fullsort(self, q, k: int):
        a = _c(q, np.uint32).reshape(-1, self.dim)
        ids = np.empty((a.shape[0], k), dtype=np.uint32)
        d2 = np.empty((a.shape[0], k), dtype=np.uint64)
        lib().ora_knn_fullsort(self._h, _p(a), a.shape[0], k, _p(ids), _p(d2))
        return ids, d2

    def range_count(self, boxes, threads: int = 0) -> np.ndarray:
        b = _c(boxes, np.uint32).reshape(-1, 2, self.dim)
        out = np.empty(b.shape[0], dtype=np.uint64)
        lib().ora_range_count(self._h, _p(b), b.shape[0], _p(out), threads)
        return out

    def range_report(self, boxes, threads: int = 0):
        """Returns (offsets[nb+1], ids) with ids ascending inside each box."""
        b = _c(boxes, np.uint32).reshape(-1, 2, self.dim)
        cnt = self.range_count(b, threads)
        off = np.zeros(b.shape[0] + 1, dtype=np.uint64)
        np.cumsum(cnt, out=off[1:])
        ids = np.empty(int(off[-1]), dtype=np.uint32)
        lib().ora_range_report(self._h, _p(b), b.shape[0], _p(off), _p(ids), threads)
        return off, ids
