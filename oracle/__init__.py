"""CPU oracle for GTS batched similarity search -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it.

Thin ctypes wrapper over ``oracle.c`` (built as ``liboracle.so`` by
``oracle/build.py``).  Everything here is marshalling; the arithmetic is in the
C file, which states what it follows in the paper:

* ``l2``/``l1``/``angular``/``edit``: the metrics (FP64 direct difference,
  FP64 sum of absolute differences, FP64 half-angle form; Wagner-Fischer).
* ``range_bf``/``knn_bf``: Definitions 1 and 2 by brute force, answers sorted
  by (distance, id), kNN answers are the first min(k, n) in that order.
* ``GtsTree``: a GTS-literal index (Algorithms 1-3) and its batched range and
  kNN searches (Algorithms 4-5), counting distance evaluations per query.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

L2, EDIT, ANGULAR, L1 = 1, 2, 3, 4


class _Set(C.Structure):
    _fields_ = [("metric", C.c_int32), ("dim", C.c_int32), ("n", C.c_int64),
                ("vecs", C.c_void_p), ("chars", C.c_void_p),
                ("offsets", C.c_void_p), ("ids", C.c_void_p)]


class _Result(C.Structure):
    _fields_ = [("nq", C.c_int64), ("offsets", C.POINTER(C.c_int64)),
                ("ids", C.POINTER(C.c_int64)), ("dist", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        L.orc_set_threads.restype = C.c_int32
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_l2.restype = C.c_double
        L.orc_l2.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
        L.orc_angular.restype = C.c_double
        L.orc_angular.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
        L.orc_l1.restype = C.c_double
        L.orc_l1.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
        L.orc_edit.restype = C.c_int32
        L.orc_edit.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64]
        L.orc_pair_distances.argtypes = [P(_Set), P(_Set), C.c_void_p]
        L.orc_range_bf.argtypes = [P(_Set), P(_Set), C.c_void_p, P(_Result)]
        L.orc_knn_bf.argtypes = [P(_Set), P(_Set), C.c_void_p, P(_Result)]
        L.orc_result_free.argtypes = [P(_Result)]
        L.orc_gts_height.restype = C.c_int32
        L.orc_gts_height.argtypes = [C.c_int64, C.c_int32]
        L.orc_gts_build.restype = C.c_void_p
        L.orc_gts_build.argtypes = [P(_Set), C.c_int32, C.c_uint64]
        L.orc_gts_free.argtypes = [C.c_void_p]
        L.orc_gts_layers.restype = C.c_int32
        L.orc_gts_layers.argtypes = [C.c_void_p]
        L.orc_gts_node_count.restype = C.c_int64
        L.orc_gts_node_count.argtypes = [C.c_void_p]
        L.orc_gts_nodes.argtypes = [C.c_void_p] + [C.c_void_p] * 5
        L.orc_gts_table.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_gts_range.argtypes = [C.c_void_p, P(_Set), C.c_void_p, C.c_int64,
                                    P(_Result), C.c_void_p]
        L.orc_gts_knn.argtypes = [C.c_void_p, P(_Set), C.c_void_p, C.c_int64,
                                  P(_Result), C.c_void_p]
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads of the brute-force loops (0: query only); returns the count
    in force."""
    return lib().orc_set_threads(int(n))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class ObjectSet:
    """A borrowed view of objects for the oracle: float32 vectors [n, dim]
    (L2, or L1 with l1=True, or the angular metric with angular=True) or
    packed strings (chars uint8, offsets int64 [n+1]) (edit), with optional
    int64 external ids (default 0..n-1)."""

    def __init__(self, vecs=None, strings=None, ids=None, angular=False, l1=False):
        if (vecs is None) == (strings is None):
            raise ValueError("give exactly one of vecs / strings")
        s = _Set()
        self._keep = []
        if vecs is not None:
            v = np.ascontiguousarray(vecs, dtype=np.float32)
            if v.ndim != 2:
                raise ValueError("vecs must be 2-D")
            self._keep.append(v)
            s.metric, s.dim, s.n = (ANGULAR if angular else L1 if l1 else L2), v.shape[1], v.shape[0]
            s.vecs = v.ctypes.data
        else:
            chars = np.ascontiguousarray(strings[0], dtype=np.uint8)
            offs = np.ascontiguousarray(strings[1], dtype=np.int64)
            if chars.size == 0:
                chars = np.zeros(1, np.uint8)
            self._keep += [chars, offs]
            s.metric, s.dim, s.n = EDIT, 0, offs.shape[0] - 1
            s.chars, s.offsets = chars.ctypes.data, offs.ctypes.data
        if ids is not None:
            idv = np.ascontiguousarray(ids, dtype=np.int64)
            if idv.shape[0] != s.n:
                raise ValueError("ids length mismatch")
            self._keep.append(idv)
            s.ids = idv.ctypes.data
        self.s = s

    @property
    def n(self):
        return self.s.n

    @property
    def metric(self):
        return self.s.metric


def _unpack(res: _Result):
    nq = res.nq
    off = np.ctypeslib.as_array(res.offsets, shape=(nq + 1,)).copy()
    total = int(off[-1])
    if total:
        ids = np.ctypeslib.as_array(res.ids, shape=(total,)).copy()
        dist = np.ctypeslib.as_array(res.dist, shape=(total,)).copy()
    else:
        ids = np.zeros(0, np.int64)
        dist = np.zeros(0, np.float64)
    lib().orc_result_free(C.byref(res))
    return [(ids[off[q]:off[q + 1]], dist[off[q]:off[q + 1]]) for q in range(nq)]


def l2(x, y) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    assert x.shape == y.shape
    return lib().orc_l2(_ptr(x), _ptr(y), x.shape[0])


def l1(x, y) -> float:
    """Manhattan distance sum |x_i - y_i| (float64)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    assert x.shape == y.shape
    return lib().orc_l1(_ptr(x), _ptr(y), x.shape[0])


def angular(x, y) -> float:
    """Angle between nonzero vectors x and y (radians, float64)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    assert x.shape == y.shape
    return lib().orc_angular(_ptr(x), _ptr(y), x.shape[0])


def edit(a: bytes, b: bytes) -> int:
    ba = np.frombuffer(a, dtype=np.uint8) if len(a) else np.zeros(1, np.uint8)
    bb = np.frombuffer(b, dtype=np.uint8) if len(b) else np.zeros(1, np.uint8)
    return lib().orc_edit(_ptr(ba), len(a), _ptr(bb), len(b))


def pair_distances(objects: ObjectSet, queries: ObjectSet) -> np.ndarray:
    out = np.empty((queries.n, objects.n), dtype=np.float64)
    lib().orc_pair_distances(C.byref(objects.s), C.byref(queries.s), _ptr(out))
    return out


def range_bf(objects: ObjectSet, queries: ObjectSet, radius):
    """Definition 1 by brute force: per query (ids, dists) with d <= r, sorted
    by (d, id).  ``radius`` is a scalar or per-query array (float64)."""
    r = np.broadcast_to(np.asarray(radius, dtype=np.float64), (queries.n,)).copy()
    res = _Result()
    lib().orc_range_bf(C.byref(objects.s), C.byref(queries.s), _ptr(r), C.byref(res))
    return _unpack(res)


def knn_bf(objects: ObjectSet, queries: ObjectSet, k):
    """Definition 2 by brute force: per query the first min(k, n) objects in
    ascending (d, id) order."""
    kv = np.broadcast_to(np.asarray(k, dtype=np.int32), (queries.n,)).copy()
    res = _Result()
    lib().orc_knn_bf(C.byref(objects.s), C.byref(queries.s), _ptr(kv), C.byref(res))
    return _unpack(res)


def gts_height(n: int, nc: int) -> int:
    return lib().orc_gts_height(n, nc)


class GtsTree:
    """GTS-literal index over an ObjectSet (Algorithms 1-3)."""

    def __init__(self, objects: ObjectSet, nc: int, seed: int = 1):
        self.objects = objects
        self.h = lib().orc_gts_build(C.byref(objects.s), nc, seed)
        if not self.h:
            raise ValueError("node capacity must be >= 2")
        self.nc = nc

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_gts_free(self.h)
            self.h = None

    @property
    def layers(self) -> int:
        return lib().orc_gts_layers(self.h)

    @property
    def node_count(self) -> int:
        return lib().orc_gts_node_count(self.h)

    def nodes(self):
        nn = self.node_count
        piv = np.empty(nn, np.int64)
        size = np.empty(nn, np.int64)
        pos = np.empty(nn, np.int64)
        mn = np.empty(nn, np.float64)
        mx = np.empty(nn, np.float64)
        lib().orc_gts_nodes(self.h, _ptr(piv), _ptr(size), _ptr(pos), _ptr(mn), _ptr(mx))
        return {"pivot": piv, "size": size, "pos": pos, "min_dis": mn, "max_dis": mx}

    def table(self):
        n = self.objects.n
        ids = np.empty(n, np.int64)
        dis = np.empty(n, np.float64)
        lib().orc_gts_table(self.h, _ptr(ids), _ptr(dis))
        return ids, dis

    def range(self, queries: ObjectSet, radius, budget: int = 0):
        """Algorithm 4; returns (answers, distance evaluations per query)."""
        r = np.broadcast_to(np.asarray(radius, dtype=np.float64), (queries.n,)).copy()
        ev = np.zeros(max(1, queries.n), np.int64)
        res = _Result()
        lib().orc_gts_range(self.h, C.byref(queries.s), _ptr(r), budget, C.byref(res), _ptr(ev))
        return _unpack(res), ev[:queries.n]

    def knn(self, queries: ObjectSet, k, budget: int = 0):
        """Algorithm 5; returns (answers, distance evaluations per query)."""
        kv = np.broadcast_to(np.asarray(k, dtype=np.int32), (queries.n,)).copy()
        ev = np.zeros(max(1, queries.n), np.int64)
        res = _Result()
        lib().orc_gts_knn(self.h, C.byref(queries.s), _ptr(kv), budget, C.byref(res), _ptr(ev))
        return _unpack(res), ev[:queries.n]
