"""Parity at the benchmark's full sizes and launch configuration.

Each whole batch runs exactly as bench.py runs it (one gts_search call), and
is then checked two ways:
  * element by element against the plain one-query-per-workgroup form over
    the whole batch (the plain form is oracle-checked on the smaller cases;
    it shares no selection or verification kernel with the batched form,
    and both report float32 direct-difference distances, so the answers
    must be identical);
  * against the oracle's brute force on a stratified sample the oracle
    finishes in seconds: random queries plus the range queries with the
    most answers (the long candidate lists that one workgroup verifies) and
    the kNN queries with the widest k-th distance.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2404_00966_amd import synth
from tests.parity import check_exact, check_knn, check_range

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RANDOM = 8      # random queries per kind
EXTREME = 4     # largest answers / widest bounds per kind


def _same(a_lists, b_lists, what):
    assert len(a_lists) == len(b_lists)
    for q, ((a, b), (c, e)) in enumerate(zip(a_lists, b_lists)):
        assert np.array_equal(a, c) and np.array_equal(b, e), (what, q, a[:6], c[:6])


def _stratified(rng, n, score, count_random=RANDOM, count_top=EXTREME):
    top = np.argsort(-np.asarray(score), kind="stable")[:count_top]
    rest = np.setdiff1d(np.arange(n), top)
    return np.concatenate([top, rng.choice(rest, count_random, replace=False)])


def test_l2_1m_d128_full_batch():
    import torch

    from paper_2404_00966_amd import gts

    w = synth.WORKLOADS["l2_1m_d128"]
    r = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))["l2_1m_d128"]["radius_f32"]
    d = synth.make_workload("l2_1m_d128")
    X = d["objects"]
    KQ, RQ = d["knn_queries"], d["range_queries"]
    print("[case] l2_1m_d128 full batch, batched and plain", flush=True)
    idx = gts.Index(torch.from_numpy(X).cuda(), gts.L2_F32, num_pivots=w["pivots"], fanout=w["fanout"],
                    leaf_size=w["leaf"], seed=w["seed"])
    Q = torch.from_numpy(np.concatenate([KQ, RQ])).cuda()
    k = np.array([w["k"]] * len(KQ) + [0] * len(RQ), np.int32)
    radius = np.full(len(KQ) + len(RQ), r, np.float32)
    res = idx.search(Q, radius=radius, k=k, result="device", flags=gts.QF_CHECK_BOUND).to_lists()
    st = idx.stats()
    print(f"[stats] batched {st}", flush=True)
    assert st["results"] == sum(len(a) for a, _ in res)
    assert st["wide_queries"] > 0, "no query reached the workgroup verification form"
    assert st["bound_violations"] == 0
    assert all(len(res[i][0]) == w["k"] for i in range(len(KQ)))
    plain = idx.search(Q, radius=radius, k=k, mode=gts.MODE_PLAIN, result="device").to_lists()
    _same(res, plain, "batched vs plain")
    sel32 = idx.search(Q, radius=radius, k=k, precision=gts.FP32, result="device").to_lists()
    print(f"[stats] float32 selection {idx.stats()}", flush=True)
    idx.close()
    _same(res, sel32, "bf16-guarded vs float32 selection")
    rng = np.random.default_rng(0)
    nk = len(KQ)
    ks = _stratified(rng, nk, [res[i][1][-1] for i in range(nk)])
    rs = _stratified(rng, len(RQ), [len(res[nk + i][0]) for i in range(len(RQ))])
    print(f"[sample] kNN {ks.tolist()} range {rs.tolist()}; most answers "
          f"{[len(res[nk + i][0]) for i in rs[:EXTREME]]}", flush=True)
    objs = O.ObjectSet(vecs=X)
    check_knn([res[i] for i in ks], O.knn_bf(objs, O.ObjectSet(vecs=KQ[ks]), w["k"]), X, KQ[ks], w["k"])
    check_range([res[nk + i] for i in rs], O.range_bf(objs, O.ObjectSet(vecs=RQ[rs]), r), X, RQ[rs], r)


def test_dna_500k_full_batch():
    import torch

    from paper_2404_00966_amd import gts

    w = synth.WORKLOADS["dna_500k"]
    d = synth.make_workload("dna_500k")
    chars, off = d["objects"]
    qc, qo = d["queries"]
    print("[case] dna_500k full batch, batched and plain", flush=True)
    idx = gts.Index((torch.from_numpy(chars).cuda(), torch.from_numpy(off).cuda()), gts.EDIT_U8,
                    num_pivots=w["pivots"], fanout=w["fanout"], seed=w["seed"])
    nq = len(qo) - 1
    Qd = (torch.from_numpy(qc).cuda(), torch.from_numpy(qo).cuda())
    res = idx.range(Qd, float(w["radius"]), result="device").to_lists()
    plain = idx.range(Qd, float(w["radius"]), mode=gts.MODE_PLAIN, result="device").to_lists()
    idx.close()
    _same(res, plain, "batched vs plain")
    rng = np.random.default_rng(1)
    sel = _stratified(rng, nq, [len(a) for a, _ in res])
    items = [qc[qo[i]:qo[i + 1]].tobytes() for i in sel]
    sc, so = synth.strings_from_bytes(items)
    ref = O.range_bf(O.ObjectSet(strings=(chars, off)), O.ObjectSet(strings=(sc, so)), float(w["radius"]))
    check_exact([res[i] for i in sel], ref)


def test_l2_4m_d96_knn_bf16():
    """4M x 96, 50,000 kNN queries (k = 32) through the bf16 MFMA path with
    float32 rechecks: the whole batch against the float32 plain path, a
    stratified sample against the float64 oracle, and the largest relative
    distance error over every returned pair of the sample."""
    import torch

    from paper_2404_00966_amd import gts

    w = synth.WORKLOADS["l2_4m_d96"]
    d = synth.make_workload("l2_4m_d96")
    X = d["objects"]
    KQ = d["knn_queries"]
    print("[case] l2_4m_d96 knn batch, batched and plain", flush=True)
    idx = gts.Index(torch.from_numpy(X).cuda(), gts.L2_F32, num_pivots=w["pivots"], fanout=w["fanout"],
                    leaf_size=w["leaf"], seed=w["seed"])
    Qd = torch.from_numpy(KQ).cuda()
    res = idx.knn(Qd, w["k"], result="device", flags=gts.QF_CHECK_BOUND).to_lists()
    st = idx.stats()
    print(f"[stats] batched {st}", flush=True)
    assert st["bound_violations"] == 0
    assert len(res) == len(KQ) and all(len(ids) == w["k"] for ids, _ in res)
    plain = idx.knn(Qd, w["k"], mode=gts.MODE_PLAIN, result="device").to_lists()
    _same(res, plain, "bf16-guarded vs float32 plain")
    sel32 = idx.knn(Qd, w["k"], precision=gts.FP32, result="device").to_lists()
    print(f"[stats] float32 selection {idx.stats()}", flush=True)
    idx.close()
    _same(res, sel32, "bf16-guarded vs float32 selection (batched)")
    rng = np.random.default_rng(2)
    ks = _stratified(rng, len(KQ), [res[i][1][-1] for i in range(len(KQ))])
    sample = [res[i] for i in ks]
    check_knn(sample, O.knn_bf(O.ObjectSet(vecs=X), O.ObjectSet(vecs=KQ[ks]), w["k"]), X, KQ[ks], w["k"])
    worst = 0.0
    for (ids, dist), q in zip(sample, KQ[ks]):
        exact = np.sqrt(((X[ids].astype(np.float64) - q.astype(np.float64)) ** 2).sum(axis=1))
        worst = max(worst, float(np.max(np.abs(dist.astype(np.float64) - exact) / np.maximum(exact, 1e-30))))
    print(f"[metric] l2_4m_d96 max relative distance error vs float64: {worst:.3e}", flush=True)
    assert worst <= 1e-5
