"""Parity at the benchmark's full sizes and launch configuration: the whole
batch runs exactly as bench.py runs it; sampled queries are checked against
the oracle's brute force (which finishes a few queries in seconds)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2404_00966_amd import synth
from tests.parity import check_exact, check_knn, check_range

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAMPLE = 12


def test_l2_1m_d128_full_batch_sampled():
    import torch

    from paper_2404_00966_amd import gts

    w = synth.WORKLOADS["l2_1m_d128"]
    r = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))["l2_1m_d128"]["radius_f32"]
    d = synth.make_workload("l2_1m_d128")
    X = d["objects"]
    KQ, RQ = d["knn_queries"], d["range_queries"]
    print("[case] l2_1m_d128 full batch", flush=True)
    idx = gts.Index(torch.from_numpy(X).cuda(), gts.L2_F32, num_pivots=w["pivots"], fanout=w["fanout"],
                    leaf_size=w["leaf"], seed=w["seed"])
    Q = np.concatenate([KQ, RQ])
    k = np.array([w["k"]] * len(KQ) + [0] * len(RQ), np.int32)
    res = idx.search(torch.from_numpy(Q).cuda(), radius=np.full(len(Q), r, np.float32), k=k).to_lists()
    st = idx.stats()
    idx.close()
    assert st["results"] == sum(len(a) for a, _ in res)
    assert all(len(res[i][0]) == w["k"] for i in range(len(KQ)))
    rng = np.random.default_rng(0)
    ks = rng.choice(len(KQ), SAMPLE, replace=False)
    rs = rng.choice(len(RQ), SAMPLE, replace=False)
    objs = O.ObjectSet(vecs=X)
    check_knn([res[i] for i in ks], O.knn_bf(objs, O.ObjectSet(vecs=KQ[ks]), w["k"]), X, KQ[ks], w["k"])
    check_range([res[len(KQ) + i] for i in rs], O.range_bf(objs, O.ObjectSet(vecs=RQ[rs]), r), X, RQ[rs], r)


def test_dna_500k_full_batch_sampled():
    import torch

    from paper_2404_00966_amd import gts

    w = synth.WORKLOADS["dna_500k"]
    d = synth.make_workload("dna_500k")
    chars, off = d["objects"]
    qc, qo = d["queries"]
    print("[case] dna_500k full batch", flush=True)
    idx = gts.Index((torch.from_numpy(chars).cuda(), torch.from_numpy(off).cuda()), gts.EDIT_U8,
                    num_pivots=w["pivots"], fanout=w["fanout"], seed=w["seed"])
    nq = len(qo) - 1
    res = idx.range((torch.from_numpy(qc).cuda(), torch.from_numpy(qo).cuda()), float(w["radius"])).to_lists()
    idx.close()
    rng = np.random.default_rng(1)
    sel = rng.choice(nq, SAMPLE, replace=False)
    items = [qc[qo[i]:qo[i + 1]].tobytes() for i in sel]
    sc, so = synth.strings_from_bytes(items)
    ref = O.range_bf(O.ObjectSet(strings=(chars, off)), O.ObjectSet(strings=(sc, so)), float(w["radius"]))
    check_exact([res[i] for i in sel], ref)


def test_l2_4m_d96_knn_bf16_sampled():
    """4M x 96, 50,000 kNN queries (k = 32) through the bf16 MFMA path with
    float32 rechecks: sampled queries against the float64 oracle, the largest
    relative distance error over every returned pair of the sample, and the
    float32 plain path on the same sample."""
    import torch

    from paper_2404_00966_amd import gts

    w = synth.WORKLOADS["l2_4m_d96"]
    d = synth.make_workload("l2_4m_d96")
    X = d["objects"]
    KQ = d["knn_queries"]
    print("[case] l2_4m_d96 knn batch", flush=True)
    idx = gts.Index(torch.from_numpy(X).cuda(), gts.L2_F32, num_pivots=w["pivots"], fanout=w["fanout"],
                    leaf_size=w["leaf"], seed=w["seed"])
    res = idx.knn(torch.from_numpy(KQ).cuda(), w["k"]).to_lists()
    assert len(res) == len(KQ) and all(len(ids) == w["k"] for ids, _ in res)
    rng = np.random.default_rng(2)
    ks = rng.choice(len(KQ), SAMPLE, replace=False)
    sample = [res[i] for i in ks]
    check_knn(sample, O.knn_bf(O.ObjectSet(vecs=X), O.ObjectSet(vecs=KQ[ks]), w["k"]), X, KQ[ks], w["k"])
    worst = 0.0
    for (ids, dist), q in zip(sample, KQ[ks]):
        exact = np.sqrt(((X[ids].astype(np.float64) - q.astype(np.float64)) ** 2).sum(axis=1))
        worst = max(worst, float(np.max(np.abs(dist.astype(np.float64) - exact) / np.maximum(exact, 1e-30))))
    print(f"[metric] l2_4m_d96 max relative distance error vs float64: {worst:.3e}", flush=True)
    assert worst <= 1e-5
    plain = idx.knn(torch.from_numpy(KQ[ks]).cuda(), w["k"], mode=gts.MODE_PLAIN).to_lists()
    idx.close()
    for (a, b), (c, e) in zip(sample, plain):
        assert np.array_equal(a, c) and np.array_equal(b, e)
