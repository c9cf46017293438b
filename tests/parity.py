"""Parity checks of GPU answers against the CPU oracle (imported by tests and
by the smoke check).

Tolerances:
  * edit distance: ids and distances identical.
  * L2: for ids in both answers the float32 distance is within 1e-5 relative
    of the oracle's float64 distance (exactly 0 when that is 0); the id sets
    may differ only by objects whose float64 distance lies within 1e-5 * r of
    the radius (range) or within 1e-5 * d_k of the oracle's k-th distance
    (kNN).  Answers are in (distance, id) order.
"""
import numpy as np

import oracle as O

REL = 1e-5


def _d64(X, q, ids):
    return np.array([O.l2(q, X[i]) for i in ids], dtype=np.float64)


def _check_sorted(ids, dist):
    for a in range(len(ids) - 1):
        assert (dist[a], ids[a]) <= (dist[a + 1], ids[a + 1]), "answer not in (distance, id) order"


def _check_common(gi, gd, ri, rd):
    ref = dict(zip(ri.tolist(), rd.tolist()))
    for i, d in zip(gi.tolist(), gd.tolist()):
        if i in ref:
            r = ref[i]
            if r == 0.0:
                assert d == 0.0, (i, d, r)
            else:
                assert abs(d - r) <= REL * r, (i, d, r)


def check_range(gpu, ref, X, Q, radius, id_to_row=None):
    """gpu/ref: per-query (ids, dist) lists; X: objects (rows by id unless
    id_to_row maps ids to rows); radius scalar or per query."""
    rad = np.broadcast_to(np.asarray(radius, np.float64), (len(ref),))
    assert len(gpu) == len(ref)
    row = (lambda i: i) if id_to_row is None else (lambda i: id_to_row[i])
    for q, ((gi, gd), (ri, rd)) in enumerate(zip(gpu, ref)):
        gi = np.asarray(gi)
        gd = np.asarray(gd, np.float64)
        assert len(set(gi.tolist())) == len(gi), "duplicate id in answer"
        _check_sorted(gi, gd)
        _check_common(gi, gd, ri, rd)
        diff = set(gi.tolist()) ^ set(ri.tolist())
        if diff:
            d = np.array([O.l2(Q[q], X[row(i)]) for i in diff])
            r = rad[q]
            assert np.all(np.abs(d - r) <= REL * max(r, 1e-30)), (q, sorted(diff)[:5], d[:5], r)


def check_knn(gpu, ref, X, Q, k, id_to_row=None):
    assert len(gpu) == len(ref)
    row = (lambda i: i) if id_to_row is None else (lambda i: id_to_row[i])
    for q, ((gi, gd), (ri, rd)) in enumerate(zip(gpu, ref)):
        gi = np.asarray(gi)
        gd = np.asarray(gd, np.float64)
        assert len(gi) == len(ri), (q, len(gi), len(ri))
        assert len(set(gi.tolist())) == len(gi), "duplicate id in answer"
        _check_sorted(gi, gd)
        _check_common(gi, gd, ri, rd)
        diff = set(gi.tolist()) ^ set(ri.tolist())
        if diff:
            dk = rd[-1]
            d = np.array([O.l2(Q[q], X[row(i)]) for i in diff])
            assert np.all(np.abs(d - dk) <= REL * max(dk, 1e-30)), (q, sorted(diff)[:5], d[:5], dk)


def check_exact(gpu, ref):
    """Edit distance: identical ids and distances."""
    assert len(gpu) == len(ref)
    for q, ((gi, gd), (ri, rd)) in enumerate(zip(gpu, ref)):
        assert np.array_equal(np.asarray(gi), ri), (q, gi[:8], ri[:8])
        assert np.array_equal(np.asarray(gd).astype(np.int64), rd.astype(np.int64)), (q, gd[:8], rd[:8])
