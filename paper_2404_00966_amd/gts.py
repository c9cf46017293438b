"""Python binding of libgts.so -- argument marshalling only.

Every stage of a search runs in the library's HIP kernels; this module turns
torch tensors / numpy arrays into the plain pointers of the C ABI
(include/gts.h) and results back into torch tensors.  torch is imported first
so the library binds to the HIP runtime torch already loaded.  There is no
fallback: if libgts.so is missing or fails to load, an error is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgts.so")

L2_F32, EDIT_U8, COSINE_F32, L1_F32 = 1, 2, 3, 4
HOST, DEVICE = 0, 1
MODE_BATCHED, MODE_PLAIN = 0, 1
QF_CHECK_BOUND, QF_NO_PRUNE = 1, 2
PRECISION_DEFAULT, BF16_GUARDED, FP32 = 0, 1, 2
STAGES = ("prep", "bound", "nodes", "cands", "group", "verify", "output", "plain")

OK, EINVAL, ENOMEM, EDEVICE, ENOTSUP = 0, -1, -2, -3, -4


class GtsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gts status {status}: {msg}")
        self.status = status


class _Objects(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int32), ("location", C.c_int32),
                ("vecs", C.c_void_p), ("chars", C.c_void_p), ("offsets", C.c_void_p)]


class _BuildOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("leaf_size", C.c_int32), ("max_strlen", C.c_int32),
                ("cache_limit", C.c_int64), ("mem_budget_bytes", C.c_int64), ("precision", C.c_int32),
                ("reserved0", C.c_int32), ("tune_cache", C.c_char_p)]


class _QueryOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("result_location", C.c_int32), ("mem_budget_bytes", C.c_int64),
                ("precision", C.c_int32), ("flags", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("nq", C.c_int64), ("total", C.c_int64), ("location", C.c_int32), ("metric", C.c_int32),
                ("offsets", C.c_void_p), ("ids", C.c_void_p), ("dist_f32", C.c_void_p),
                ("dist_i32", C.c_void_p), ("priv", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("nq", C.c_int64), ("node_tests", C.c_int64), ("leaf_pairs", C.c_int64),
                ("tile_pairs", C.c_int64), ("candidates", C.c_int64), ("verified", C.c_int64),
                ("results", C.c_int64), ("ms_total", C.c_double), ("ms_stage", C.c_double * 8),
                ("groups", C.c_int64), ("bound_window", C.c_int64), ("tuning", C.c_int64),
                ("bound_evals", C.c_int64), ("wide_queries", C.c_int64), ("bound_violations", C.c_int64),
                ("own_pairs", C.c_int64), ("filter_objects", C.c_int64), ("sweep_grid_per_cu", C.c_int64),
                ("group_retries", C.c_int64), ("max_query_candidates", C.c_int64)]


class _Info(C.Structure):
    _fields_ = [("metric", C.c_int32), ("dim", C.c_int32), ("num_pivots", C.c_int32), ("fanout", C.c_int32),
                ("levels", C.c_int32), ("max_strlen", C.c_int32), ("n_indexed", C.c_int64),
                ("n_live", C.c_int64), ("n_cache", C.c_int64), ("n_nodes", C.c_int64),
                ("n_leaves", C.c_int64), ("n_slabs", C.c_int64), ("rebuilds", C.c_int64),
                ("device_bytes", C.c_int64), ("rebuild_ms", C.c_double), ("epoch", C.c_int64)]


REQ_RANGE, REQ_KNN, REQ_INSERT, REQ_DELETE = 1, 2, 3, 4


class _Request(C.Structure):
    _fields_ = [("index", C.c_int32), ("kind", C.c_int32), ("objects", _Objects), ("radius", C.c_float),
                ("k", C.c_int32), ("ids", C.c_void_p), ("n_ids", C.c_int64), ("tag", C.c_uint64)]


class _Completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("tag", C.c_uint64), ("kind", C.c_int32), ("status", C.c_int32),
                ("error", C.c_char_p), ("result", _Result), ("new_ids", C.c_void_p), ("count", C.c_int64),
                ("batch", C.c_int64), ("t_submit_ms", C.c_double), ("t_start_ms", C.c_double),
                ("t_done_ms", C.c_double), ("priv", C.c_void_p)]


class _ServerOpts(C.Structure):
    _fields_ = [("lanes_per_index", C.c_int32), ("max_batch_queries", C.c_int32),
                ("mem_budget_bytes", C.c_int64), ("keep_results", C.c_int32)]


class _ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("queries", C.c_int64), ("batches", C.c_int64), ("updates", C.c_int64),
                ("mean_batch_queries", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("max_ms", C.c_double), ("span_ms", C.c_double)]


class _PlanIO(C.Structure):
    _fields_ = [("queries", C.c_void_p), ("radius", C.c_void_p), ("k", C.c_void_p), ("offsets", C.c_void_p),
                ("ids", C.c_void_p), ("dist", C.c_void_p), ("status", C.c_void_p)]


PLAN_BAD_INPUT, PLAN_BAD_QUERY, PLAN_CANDIDATES, PLAN_ANSWERS = 1, 2, 4, 8


EXPORTS = ("gts_build_index", "gts_range_query", "gts_knn_query", "gts_search", "gts_insert", "gts_delete",
           "gts_result_copy", "gts_result_free", "gts_destroy", "gts_get_info", "gts_get_stats",
           "gts_set_timing", "gts_last_error", "gts_server_create", "gts_server_submit", "gts_server_replay",
           "gts_server_poll", "gts_server_release", "gts_server_flush", "gts_server_get_stats",
           "gts_server_destroy", "gts_update_batch", "gts_cost_model", "gts_choose_fanout", "gts_search_noalloc",
           "gts_plan_create", "gts_plan_launch", "gts_plan_destroy")

_lib = None


def library():
    """Load libgts.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.gts_build_index.argtypes = [P(_Objects), C.c_int32, C.c_int32, C.c_int32, P(_BuildOpts), C.c_void_p,
                                      P(C.c_void_p)]
        L.gts_search.argtypes = [C.c_void_p, P(_Objects), C.c_void_p, C.c_void_p, P(_QueryOpts), P(_Result)]
        L.gts_range_query.argtypes = [C.c_void_p, P(_Objects), C.c_void_p, P(_QueryOpts), P(_Result)]
        L.gts_knn_query.argtypes = [C.c_void_p, P(_Objects), C.c_void_p, P(_QueryOpts), P(_Result)]
        L.gts_insert.argtypes = [C.c_void_p, P(_Objects), C.c_void_p]
        L.gts_delete.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, P(C.c_int64)]
        L.gts_cost_model.restype = C.c_double
        L.gts_cost_model.argtypes = [C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_double]
        L.gts_choose_fanout.argtypes = [P(_Objects), C.c_int32, C.c_float, C.c_double, P(C.c_int32), C.c_void_p]
        L.gts_update_batch.argtypes = [C.c_void_p, P(_Objects), C.c_void_p, C.c_int64, C.c_void_p, P(C.c_int64)]
        L.gts_result_copy.argtypes = [P(_Result), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.gts_result_free.argtypes = [P(_Result)]
        L.gts_destroy.argtypes = [C.c_void_p]
        L.gts_get_info.argtypes = [C.c_void_p, P(_Info)]
        L.gts_get_stats.argtypes = [C.c_void_p, P(_Stats)]
        L.gts_set_timing.argtypes = [C.c_void_p, C.c_int32]
        L.gts_server_create.argtypes = [C.c_void_p, C.c_int32, P(_ServerOpts), P(C.c_void_p)]
        L.gts_server_submit.argtypes = [C.c_void_p, P(_Request), P(C.c_uint64)]
        L.gts_server_replay.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.gts_server_poll.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, P(C.c_int32)]
        L.gts_server_release.argtypes = [P(_Completion)]
        L.gts_server_flush.argtypes = [C.c_void_p]
        L.gts_server_get_stats.argtypes = [C.c_void_p, P(_ServerStats)]
        L.gts_server_destroy.argtypes = [C.c_void_p]
        L.gts_search_noalloc.argtypes = [C.c_void_p, P(_Objects), C.c_void_p, C.c_void_p, P(_QueryOpts),
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, P(C.c_int64)]
        L.gts_plan_create.argtypes = [C.c_void_p, C.c_int64, C.c_int64, P(_QueryOpts), P(_PlanIO), P(C.c_void_p)]
        L.gts_plan_launch.argtypes = [C.c_void_p, C.c_void_p]
        L.gts_plan_destroy.argtypes = [C.c_void_p]
        L.gts_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("gts_last_error", "gts_cost_model"):
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        raise GtsError(status, library().gts_last_error().decode())


class _Keep(list):
    """Holds tensors alive for the duration of a call."""


def _objects(data, metric, keep: _Keep) -> _Objects:
    """torch tensor / numpy array (L2: [n, dim] float32) or (chars, offsets)
    pair (EDIT) -> gts_objects.  CUDA tensors are passed as device pointers."""
    o = _Objects()
    if metric != EDIT_U8:
        t = data if isinstance(data, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(data))
        t = t.to(torch.float32).contiguous()
        if t.dim() != 2:
            raise ValueError("L2 objects must be a 2-D [n, dim] tensor")
        keep.append(t)
        o.n, o.dim = t.shape[0], t.shape[1]
        o.location = DEVICE if t.is_cuda else HOST
        o.vecs = t.data_ptr() if t.numel() else None
    else:
        chars, offsets = data
        ct = chars if isinstance(chars, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(chars, np.uint8))
        ot = offsets if isinstance(offsets, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(offsets, np.int64))
        ct = ct.to(torch.uint8).contiguous()
        ot = ot.to(torch.int64).contiguous()
        if ct.numel() == 0:
            ct = torch.zeros(1, dtype=torch.uint8, device=ot.device)
        keep += [ct, ot]
        o.n = ot.shape[0] - 1
        o.location = DEVICE if ot.is_cuda else HOST
        o.chars = ct.data_ptr()
        o.offsets = ot.data_ptr()
    return o


class Result:
    """CSR answers: query i's entries are offsets[i]:offsets[i+1] of ids/dist."""

    def __init__(self, offsets, ids, dist):
        self.offsets, self.ids, self.dist = offsets, ids, dist

    def __len__(self):
        return self.offsets.shape[0] - 1

    def query(self, i):
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        return self.ids[a:b], self.dist[a:b]

    def to_lists(self):
        off = self.offsets.cpu().numpy()
        ids = self.ids.cpu().numpy()
        dist = self.dist.cpu().numpy()
        return [(ids[off[q]:off[q + 1]], dist[off[q]:off[q + 1]]) for q in range(len(off) - 1)]


def cost_model(n, fanout, sigma2, radius, concurrency):
    """gts_cost_model: the range-query cost bound of the paper's cost model."""
    return library().gts_cost_model(int(n), int(fanout), float(sigma2), float(radius), float(concurrency))


def choose_fanout(objects, metric, radius, concurrency=0.0):
    """gts_choose_fanout: (best fanout, model costs of fanouts 2..64)."""
    keep = _Keep()
    o = _objects(objects, metric, keep)
    best = C.c_int32(0)
    costs = np.zeros(63, np.float64)
    _check(library().gts_choose_fanout(C.byref(o), metric, float(radius), float(concurrency), C.byref(best),
                                       costs.ctypes.data))
    return best.value, costs


class Index:
    """A GTS index in GPU memory (see include/gts.h for the semantics)."""

    def __init__(self, objects, metric=L2_F32, num_pivots=8, fanout=8, leaf_size=0, seed=0, cache_limit=0,
                 mem_budget_bytes=0, max_strlen=0, stream=None, precision=PRECISION_DEFAULT, tune_cache=None):
        L = library()
        self.metric = metric
        keep = _Keep()
        o = _objects(objects, metric, keep)
        opts = _BuildOpts(seed, leaf_size, max_strlen, cache_limit, mem_budget_bytes, precision, 0,
                          None if tune_cache is None else os.fsencode(tune_cache))
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        self._stream = stream
        sptr = stream.cuda_stream if stream is not None else None
        h = C.c_void_p()
        _check(L.gts_build_index(C.byref(o), metric, num_pivots, fanout, C.byref(opts), sptr, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            library().gts_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries ------------------------------------------------------------
    def search(self, queries, radius=None, k=None, mode=MODE_BATCHED, result="auto", mem_budget_bytes=0,
               precision=PRECISION_DEFAULT, flags=0):
        """Mixed batch: query i is kNN when k[i] > 0, else range with radius[i]."""
        L = library()
        keep = _Keep()
        o = _objects(queries, self.metric, keep)
        nq = o.n
        r_arr = None if radius is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(radius, np.float32), (nq,)))
        k_arr = None if k is None else np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
        if result == "auto":
            rloc = o.location
        else:
            rloc = DEVICE if result == "device" else HOST
        qo = _QueryOpts(mode, rloc, mem_budget_bytes, precision, flags)
        res = _Result()
        _check(L.gts_search(self._h, C.byref(o), None if r_arr is None else r_arr.ctypes.data,
                            None if k_arr is None else k_arr.ctypes.data, C.byref(qo), C.byref(res)))
        try:
            dev = torch.device("cuda") if rloc == DEVICE else torch.device("cpu")
            off = torch.empty(nq + 1, dtype=torch.int64, device=dev)
            ids = torch.empty(max(res.total, 0), dtype=torch.int64, device=dev)
            dt = torch.int32 if self.metric == EDIT_U8 else torch.float32
            dist = torch.empty(max(res.total, 0), dtype=dt, device=dev)
            if rloc == DEVICE:
                torch.cuda.current_stream().synchronize()
            _check(L.gts_result_copy(C.byref(res), rloc, off.data_ptr(), ids.data_ptr() if res.total else None,
                                     dist.data_ptr() if res.total else None))
        finally:
            L.gts_result_free(C.byref(res))
        return Result(off, ids, dist)

    def search_noalloc(self, queries, radius=None, k=None, capacity=None, precision=PRECISION_DEFAULT):
        """gts_search_noalloc: device queries, answers written into output
        tensors allocated here (the library call itself allocates nothing).
        Returns (Result, total).  capacity defaults to 64 answers per query."""
        L = library()
        keep = _Keep()
        o = _objects(queries, self.metric, keep)
        nq = o.n
        r_arr = None if radius is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(radius, np.float32), (nq,)))
        k_arr = None if k is None else np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
        cap = 64 * max(nq, 1) if capacity is None else int(capacity)
        dev = torch.device("cuda")
        off = torch.empty(nq + 1, dtype=torch.int64, device=dev)
        ids = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
        dt = torch.int32 if self.metric == EDIT_U8 else torch.float32
        dist = torch.empty(max(cap, 1), dtype=dt, device=dev)
        total = C.c_int64(0)
        qo = _QueryOpts(MODE_BATCHED, DEVICE, 0, precision, 0)
        torch.cuda.current_stream().synchronize()
        _check(L.gts_search_noalloc(self._h, C.byref(o), None if r_arr is None else r_arr.ctypes.data,
                                    None if k_arr is None else k_arr.ctypes.data, C.byref(qo), off.data_ptr(),
                                    ids.data_ptr(), dist.data_ptr(), cap, C.byref(total)))
        return Result(off, ids[:total.value], dist[:total.value]), total.value

    def range(self, queries, radius, **kw):
        return self.search(queries, radius=radius, k=None, **kw)

    def knn(self, queries, k, **kw):
        return self.search(queries, radius=None, k=k, **kw)

    # -- updates ------------------------------------------------------------
    def insert(self, objects):
        keep = _Keep()
        o = _objects(objects, self.metric, keep)
        ids = np.zeros(max(o.n, 1), np.int64)
        _check(library().gts_insert(self._h, C.byref(o), ids.ctypes.data))
        return ids[:o.n]

    def delete(self, ids):
        a = np.ascontiguousarray(np.asarray(ids, np.int64).reshape(-1))
        n = C.c_int64(0)
        _check(library().gts_delete(self._h, a.ctypes.data if a.size else None, a.size, C.byref(n)))
        return n.value

    def update_batch(self, objects=None, delete_ids=()):
        """Delete ids and insert objects together, then rebuild (returns the
        new ids and the number of ids deleted)."""
        keep = _Keep()
        o = _objects(objects, self.metric, keep) if objects is not None else None
        n_new = o.n if o is not None else 0
        ids = np.zeros(max(n_new, 1), np.int64)
        d = np.ascontiguousarray(np.asarray(delete_ids, np.int64).reshape(-1))
        nd = C.c_int64(0)
        _check(library().gts_update_batch(self._h, C.byref(o) if o is not None else None,
                                          d.ctypes.data if d.size else None, d.size, ids.ctypes.data,
                                          C.byref(nd)))
        return ids[:n_new], nd.value

    # -- inspection ----------------------------------------------------------
    def info(self):
        i = _Info()
        _check(library().gts_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in _Info._fields_}

    def stats(self):
        s = _Stats()
        _check(library().gts_get_stats(self._h, C.byref(s)))
        d = {f: getattr(s, f) for f, _ in _Stats._fields_ if f != "ms_stage"}
        d["ms_stage"] = {STAGES[i]: s.ms_stage[i] for i in range(8)}
        return d

    def set_timing(self, on=True):
        _check(library().gts_set_timing(self._h, 1 if on else 0))


class Plan:
    """gts_plan_*: a batched search of nq device queries on a vector index,
    recorded once into a HIP graph and replayed.  The plan's input tensors
    (queries [nq, dim], radius [nq], k [nq]; k == 0 marks a range query) are
    filled in place before launch(); the answers (offsets, ids, dist) and the
    status word are read after it, in stream order."""

    def __init__(self, index, nq, capacity, precision=PRECISION_DEFAULT, mem_budget_bytes=0, flags=0):
        L = library()
        dim = index.info()["dim"]
        dev = torch.device("cuda")
        self.index = index
        self.nq, self.capacity = int(nq), int(capacity)
        self.queries = torch.zeros((self.nq, dim), dtype=torch.float32, device=dev)
        self.radius = torch.zeros(self.nq, dtype=torch.float32, device=dev)
        self.k = torch.zeros(self.nq, dtype=torch.int32, device=dev)
        self.offsets = torch.zeros(self.nq + 1, dtype=torch.int64, device=dev)
        self.ids = torch.zeros(max(self.capacity, 1), dtype=torch.int64, device=dev)
        self.dist = torch.zeros(max(self.capacity, 1), dtype=torch.float32, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        io = _PlanIO(self.queries.data_ptr(), self.radius.data_ptr(), self.k.data_ptr(), self.offsets.data_ptr(),
                     self.ids.data_ptr(), self.dist.data_ptr(), self.status.data_ptr())
        qo = _QueryOpts(MODE_BATCHED, DEVICE, int(mem_budget_bytes), precision, int(flags))
        torch.cuda.current_stream().synchronize()
        h = C.c_void_p()
        _check(L.gts_plan_create(index._h, self.nq, self.capacity, C.byref(qo), C.byref(io), C.byref(h)))
        self._h = h

    def launch(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(library().gts_plan_launch(self._h, s.cuda_stream))

    def result(self):
        """(Result, status) of the last launch (waits for the current stream)."""
        torch.cuda.current_stream().synchronize()
        st = int(self.status.item())
        total = int(self.offsets[-1].item())
        n = min(total, self.capacity)
        return Result(self.offsets.clone(), self.ids[:n].clone(), self.dist[:n].clone()), st

    def close(self):
        if getattr(self, "_h", None):
            library().gts_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over built indexes (include/gts.h,
    gts_server_*).  Requests: ("range", index_no, queries, r),
    ("knn", index_no, queries, k), ("insert", index_no, objects),
    ("delete", index_no, ids).  Completions come back as dicts with host
    numpy answers; a query request's answers are a list of (ids, dist) per
    query of the request."""

    def __init__(self, indexes, lanes_per_index=2, max_batch_queries=16384, mem_budget_bytes=0,
                 keep_results=True):
        L = library()
        self._indexes = list(indexes)
        self._metrics = [ix.metric for ix in self._indexes]
        arr = (C.c_void_p * len(self._indexes))(*[ix._h.value for ix in self._indexes])
        opts = _ServerOpts(lanes_per_index, max_batch_queries, mem_budget_bytes, 1 if keep_results else 0)
        h = C.c_void_p()
        _check(L.gts_server_create(arr, len(self._indexes), C.byref(opts), C.byref(h)))
        self._h = h

    def _request(self, req, keep):
        kind, index_no = req[0], req[1]
        r = _Request()
        r.index = index_no
        # an index number out of range is the library's to reject
        metric = self._metrics[index_no] if 0 <= index_no < len(self._metrics) else self._metrics[0]
        if kind == "range":
            r.kind, r.objects, r.radius = REQ_RANGE, _objects(req[2], metric, keep), float(req[3])
        elif kind == "knn":
            r.kind, r.objects, r.k = REQ_KNN, _objects(req[2], metric, keep), int(req[3])
        elif kind == "insert":
            r.kind, r.objects = REQ_INSERT, _objects(req[2], metric, keep)
        elif kind == "delete":
            a = np.ascontiguousarray(np.asarray(req[2], np.int64).reshape(-1))
            keep.append(a)
            r.kind, r.ids, r.n_ids = REQ_DELETE, (a.ctypes.data if a.size else None), a.size
        else:
            raise ValueError(f"unknown request kind {kind!r}")
        r.tag = int(req[4]) if len(req) > 4 else 0
        return r

    def submit(self, req):
        """Queue one request tuple; returns its ticket."""
        keep = _Keep()
        r = self._request(req, keep)
        t = C.c_uint64(0)
        _check(library().gts_server_submit(self._h, C.byref(r), C.byref(t)))
        return t.value

    def replay(self, reqs, arrival_ms):
        """Open-loop replay: submit reqs[i] at arrival_ms[i] after the call
        starts (the library sleeps between submissions).  Returns tickets."""
        keep = _Keep()
        arr = (_Request * len(reqs))(*[self._request(q, keep) for q in reqs])
        t = np.ascontiguousarray(np.asarray(arrival_ms, np.float64))
        tickets = np.zeros(max(len(reqs), 1), np.uint64)
        _check(library().gts_server_replay(self._h, C.addressof(arr), t.ctypes.data, len(reqs),
                                           tickets.ctypes.data))
        return tickets[:len(reqs)]

    def poll(self, max_items=256, wait_ms=-1):
        """Take up to max_items completions (wait_ms < 0: until one is ready
        or nothing is pending)."""
        L = library()
        buf = (_Completion * max_items)()
        n = C.c_int32(0)
        _check(L.gts_server_poll(self._h, C.addressof(buf), max_items, wait_ms, C.byref(n)))
        out = []
        for i in range(n.value):
            c = buf[i]
            d = {"ticket": c.ticket, "tag": c.tag, "kind": c.kind, "status": c.status,
                 "error": (c.error or b"").decode(), "batch": c.batch, "count": c.count,
                 "t_submit_ms": c.t_submit_ms, "t_start_ms": c.t_start_ms, "t_done_ms": c.t_done_ms}
            if c.status == OK and c.kind in (REQ_RANGE, REQ_KNN):
                res = c.result
                nq = res.nq
                off = np.ctypeslib.as_array(C.cast(res.offsets, C.POINTER(C.c_int64)), (nq + 1,)).copy()
                tot = int(res.total)
                ids = np.ctypeslib.as_array(C.cast(res.ids, C.POINTER(C.c_int64)), (tot,)).copy() if tot else \
                    np.zeros(0, np.int64)
                if res.metric != EDIT_U8:
                    dist = np.ctypeslib.as_array(C.cast(res.dist_f32, C.POINTER(C.c_float)), (tot,)).copy() \
                        if tot else np.zeros(0, np.float32)
                else:
                    dist = np.ctypeslib.as_array(C.cast(res.dist_i32, C.POINTER(C.c_int32)), (tot,)).copy() \
                        if tot else np.zeros(0, np.int32)
                d["answers"] = [(ids[off[q]:off[q + 1]], dist[off[q]:off[q + 1]]) for q in range(nq)]
            if c.status == OK and c.kind == REQ_INSERT and c.count:
                d["new_ids"] = np.ctypeslib.as_array(C.cast(c.new_ids, C.POINTER(C.c_int64)), (c.count,)).copy()
            L.gts_server_release(C.byref(c))
            out.append(d)
        return out

    def flush(self):
        _check(library().gts_server_flush(self._h))

    def stats(self):
        s = _ServerStats()
        _check(library().gts_server_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            library().gts_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
