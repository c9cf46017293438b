"""Parity checks of GPU answers against the CPU oracle (imported by tests and
by the smoke check).

Tolerances:
  * edit distance: ids and distances identical.
  * L2: for ids in both answers the float32 distance is within 1e-5 relative
    of the oracle's float64 distance (exactly 0 when that is 0); the id sets
    may differ only by objects whose float64 distance lies within 1e-5 * r of
    the radius (range) or within 1e-5 * d_k of the oracle's k-th distance
    (kNN).  Answers are in (distance, id) order.
  * L1 (Manhattan): as L2 with the relative tolerance max(1e-5, (D + 2) 2^-24)
    (L1_TOL_FOR(D)).
  * angular (cosine): the same with the tolerance ANGULAR_TOL(theta) =
    (1e-5 * theta + 1e-6) / cos(theta / 2): the library measures the float32
    chord d between unit vectors rounded to float (each within one rounding,
    2^-24, of the true unit vector) and reports 2 asin(d / 2), whose error is
    at most (2 * 2^-24 + (D/2 + 2) 2^-24 d) / cos(theta / 2) plus a few
    roundings of theta; for D <= 128 that is inside ANGULAR_TOL.
"""
import numpy as np

import oracle as O

REL = 1e-5


def L2_TOL(d):
    return REL * d


def L1_TOL_FOR(dim):
    """Manhattan: every |x_i - y_i| is within one float32 rounding and any
    float32 summation order of D terms adds at most (D - 1) 2^-24 of the sum
    (the cache-list tile sums in coordinate order); for D beyond about 160
    that exceeds the L2 tolerance, so the tolerance is the larger of the two."""
    rel = max(REL, (dim + 2) * 2.0 ** -24)
    return lambda d: rel * d


def ANGULAR_TOL(t):
    return (REL * t + 1e-6) / max(np.cos(t / 2.0), 1e-3)


def _check_sorted(ids, dist):
    for a in range(len(ids) - 1):
        assert (dist[a], ids[a]) <= (dist[a + 1], ids[a + 1]), "answer not in (distance, id) order"


def _check_common(gi, gd, ri, rd, tol):
    ref = dict(zip(ri.tolist(), rd.tolist()))
    for i, d in zip(gi.tolist(), gd.tolist()):
        if i in ref:
            r = ref[i]
            if r == 0.0 and tol is L2_TOL:
                assert d == 0.0, (i, d, r)
            else:
                assert abs(d - r) <= tol(r), (i, d, r)


def check_range(gpu, ref, X, Q, radius, id_to_row=None, dist=O.l2, tol=L2_TOL):
    """gpu/ref: per-query (ids, dist) lists; X: objects (rows by id unless
    id_to_row maps ids to rows); radius scalar or per query; dist / tol: the
    oracle's metric and the tolerance at a distance."""
    rad = np.broadcast_to(np.asarray(radius, np.float64), (len(ref),))
    assert len(gpu) == len(ref)
    row = (lambda i: i) if id_to_row is None else (lambda i: id_to_row[i])
    for q, ((gi, gd), (ri, rd)) in enumerate(zip(gpu, ref)):
        gi = np.asarray(gi)
        gd = np.asarray(gd, np.float64)
        assert len(set(gi.tolist())) == len(gi), "duplicate id in answer"
        _check_sorted(gi, gd)
        _check_common(gi, gd, ri, rd, tol)
        diff = set(gi.tolist()) ^ set(ri.tolist())
        if diff:
            d = np.array([dist(Q[q], X[row(i)]) for i in diff])
            r = rad[q]
            assert np.all(np.abs(d - r) <= max(tol(r), 1e-30)), (q, sorted(diff)[:5], d[:5], r)


def check_knn(gpu, ref, X, Q, k, id_to_row=None, dist=O.l2, tol=L2_TOL):
    assert len(gpu) == len(ref)
    row = (lambda i: i) if id_to_row is None else (lambda i: id_to_row[i])
    for q, ((gi, gd), (ri, rd)) in enumerate(zip(gpu, ref)):
        gi = np.asarray(gi)
        gd = np.asarray(gd, np.float64)
        assert len(gi) == len(ri), (q, len(gi), len(ri))
        assert len(set(gi.tolist())) == len(gi), "duplicate id in answer"
        _check_sorted(gi, gd)
        _check_common(gi, gd, ri, rd, tol)
        diff = set(gi.tolist()) ^ set(ri.tolist())
        if diff:
            dk = rd[-1]
            d = np.array([dist(Q[q], X[row(i)]) for i in diff])
            assert np.all(np.abs(d - dk) <= max(tol(dk), 1e-30)), (q, sorted(diff)[:5], d[:5], dk)


def check_exact(gpu, ref):
    """Edit distance: identical ids and distances."""
    assert len(gpu) == len(ref)
    for q, ((gi, gd), (ri, rd)) in enumerate(zip(gpu, ref)):
        gi = np.asarray(gi)
        if not np.array_equal(gi, ri):
            extra = sorted(set(gi.tolist()) - set(ri.tolist()))
            missing = sorted(set(ri.tolist()) - set(gi.tolist()))
            raise AssertionError(f"query {q}: {len(gi)} ids vs {len(ri)} expected; extra {extra[:12]}, "
                                 f"missing {missing[:12]}; got {list(zip(gi.tolist(), np.asarray(gd).tolist()))[:40]}, "
                                 f"expected {list(zip(ri.tolist(), rd.tolist()))[:40]}")
        assert np.array_equal(np.asarray(gd).astype(np.int64), rd.astype(np.int64)), (q, gd[:8], rd[:8])
