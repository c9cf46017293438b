"""The angular metric (cosine similarity; GTS_COSINE_F32) through the C ABI
against the oracle's float64 angle (tolerance ANGULAR_TOL of tests/parity.py),
in the batched form (bf16 and float32 selection) and the plain form, which
must agree exactly with one another; rows wider than the MFMA path; streamed
updates with scaled copies (same direction, angle 0); zero vectors refused."""
import numpy as np
import pytest

import oracle as O
from paper_2404_00966_amd import synth
from tests.parity import ANGULAR_TOL, check_knn, check_range

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gts():
    import torch

    from paper_2404_00966_amd import gts as g

    assert torch.cuda.is_available()
    g.library()
    return g


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _lists_equal(a, b):
    for (i1, d1), (i2, d2) in zip(a, b):
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2)


def _radius(X, Q, count):
    D = O.pair_distances(O.ObjectSet(vecs=X, angular=True), O.ObjectSet(vecs=Q, angular=True))
    return float(np.float32(np.sort(D.ravel())[count]))


@pytest.mark.parametrize("dim", [48, 128])
def test_angular_forms_agree_and_match_oracle(gts, dim):
    d = synth.gaussian_mixture(400 + dim, 12000, dim, 15, -4.0, 4.0, 1.0, 120, 120)
    X = d["objects"]
    RQ, KQ = d["range_queries"], d["knn_queries"]
    r = _radius(X, RQ, 120 * 40)
    _say(f"angular dim={dim} r={r}")
    idx = gts.Index(_dev(X), gts.COSINE_F32, num_pivots=8, fanout=8, leaf_size=64, seed=4)
    assert idx.info()["metric"] == gts.COSINE_F32
    Q = _dev(np.concatenate([RQ, KQ]))
    k = np.array([0] * 120 + [11] * 120, np.int32)
    radius = np.full(240, r, np.float32)
    a = idx.search(Q, radius=radius, k=k, flags=gts.QF_CHECK_BOUND).to_lists()
    assert idx.stats()["bound_violations"] == 0
    b = idx.search(Q, radius=radius, k=k, precision=gts.FP32).to_lists()
    c = idx.search(Q, radius=radius, k=k, mode=gts.MODE_PLAIN).to_lists()
    idx.close()
    _lists_equal(a, b)
    _lists_equal(a, c)
    objs = O.ObjectSet(vecs=X, angular=True)
    check_range(a[:120], O.range_bf(objs, O.ObjectSet(vecs=RQ, angular=True), r), X, RQ, r,
                dist=O.angular, tol=ANGULAR_TOL)
    check_knn(a[120:], O.knn_bf(objs, O.ObjectSet(vecs=KQ, angular=True), 11), X, KQ, 11,
              dist=O.angular, tol=ANGULAR_TOL)


def test_angular_wide_rows(gts):
    """300-d rows (beyond the MFMA path) take the float32 path."""
    d = synth.gaussian_mixture(410, 4000, 300, 6, -3.0, 3.0, 1.0, 30, 30)
    X, RQ, KQ = d["objects"], d["range_queries"], d["knn_queries"]
    r = _radius(X, RQ, 30 * 25)
    _say(f"angular dim=300 r={r}")
    idx = gts.Index(_dev(X), gts.COSINE_F32, num_pivots=6, fanout=4, leaf_size=64, seed=5)
    res = idx.search(_dev(np.concatenate([RQ, KQ])), radius=np.full(60, r, np.float32),
                     k=np.array([0] * 30 + [9] * 30, np.int32)).to_lists()
    idx.close()
    objs = O.ObjectSet(vecs=X, angular=True)
    check_range(res[:30], O.range_bf(objs, O.ObjectSet(vecs=RQ, angular=True), r), X, RQ, r,
                dist=O.angular, tol=ANGULAR_TOL)
    check_knn(res[30:], O.knn_bf(objs, O.ObjectSet(vecs=KQ, angular=True), 9), X, KQ, 9,
              dist=O.angular, tol=ANGULAR_TOL)


def test_angular_updates_and_scaled_copies(gts):
    d = synth.gaussian_mixture(420, 5000, 32, 8, -4.0, 4.0, 1.0, 60, 60)
    X, RQ, KQ = d["objects"], d["range_queries"], d["knn_queries"]
    _say("angular updates")
    idx = gts.Index(_dev(X), gts.COSINE_F32, num_pivots=6, fanout=6, leaf_size=32, seed=6, cache_limit=10000)
    # scaled copies of some queries (angle 0 to the query) and of some objects
    extra = np.concatenate([RQ[:10] * np.float32(3.0), X[:20] * np.float32(0.25)]).astype(np.float32)
    new_ids = idx.insert(extra)
    assert len(new_ids) == 30
    gone = np.arange(0, 5000, 7)
    assert idx.delete(gone) == len(gone)
    live = np.ones(5000 + 30, bool)
    live[gone] = False
    allx = np.concatenate([X, extra])
    keep_ids = np.nonzero(live)[0]
    objs = O.ObjectSet(vecs=allx[keep_ids], ids=keep_ids, angular=True)
    r = _radius(allx[keep_ids], RQ, 60 * 20)
    Q = _dev(np.concatenate([RQ, KQ]))
    res = idx.search(Q, radius=np.full(120, r, np.float32), k=np.array([0] * 60 + [15] * 60, np.int32)).to_lists()
    idx.close()
    row = {int(i): int(j) for j, i in enumerate(keep_ids)}
    Xk = allx[keep_ids]
    check_range(res[:60], O.range_bf(objs, O.ObjectSet(vecs=RQ, angular=True), r), Xk, RQ, r, id_to_row=row,
                dist=O.angular, tol=ANGULAR_TOL)
    check_knn(res[60:], O.knn_bf(objs, O.ObjectSet(vecs=KQ, angular=True), 15), Xk, KQ, 15, id_to_row=row,
              dist=O.angular, tol=ANGULAR_TOL)
    # the scaled copies of the first range queries are at angle ~0
    for q in range(10):
        ids, dist = res[q]
        assert int(new_ids[q]) in ids.tolist()
        assert dist[ids.tolist().index(int(new_ids[q]))] <= 1e-3


def test_angular_zero_vectors_refused(gts):
    X = np.random.default_rng(7).standard_normal((200, 8)).astype(np.float32)
    _say("angular zero vectors")
    bad = X.copy()
    bad[17] = 0.0
    with pytest.raises(gts.GtsError):
        gts.Index(_dev(bad), gts.COSINE_F32, num_pivots=4, fanout=4)
    idx = gts.Index(_dev(X), gts.COSINE_F32, num_pivots=4, fanout=4)
    Q = X[:5].copy()
    Q[2] = 0.0
    with pytest.raises(gts.GtsError):
        idx.knn(_dev(Q), 3)
    with pytest.raises(gts.GtsError):
        idx.insert(np.zeros((1, 8), np.float32))
    res = idx.knn(_dev(X[:5]), 3).to_lists()     # still usable
    assert all(len(i) == 3 for i, _ in res)
    idx.close()
