"""Search plans (gts_plan_*: a fixed-shape batch recorded into a HIP graph)
through the C ABI against gts_search on the same index and inputs: identical
answers (offsets, ids, distances, element by element) on every replay, with
the query contents changed in place between replays and eager work on the
stream in between; after updates and a rebuild (the plan records its graph
again); for the Euclidean, Manhattan and angular metrics; the status flags
(bad inputs, bad queries, candidate and answer overflow); one replay against
the oracle's brute force."""
import numpy as np
import pytest

import oracle as O
from paper_2404_00966_amd import synth
from tests.parity import check_knn, check_range

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


def _same(res_a, res_b):
    a, b = res_a.to_lists(), res_b.to_lists()
    assert len(a) == len(b)
    for q, ((i1, d1), (i2, d2)) in enumerate(zip(a, b)):
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2), (q, i1[:5], i2[:5], d1[:5], d2[:5])


def _fill(plan, q, r, k):
    plan.queries.copy_(_dev(q))
    plan.radius.copy_(_dev(r))
    plan.k.copy_(_dev(k))


def _inputs(rng, pool, nq, r_lo, r_hi, kmax):
    q = pool[rng.choice(len(pool), nq, replace=False)]
    k = np.where(rng.random(nq) < 0.5, rng.integers(1, kmax + 1, nq), 0).astype(np.int32)
    r = rng.uniform(r_lo, r_hi, nq).astype(np.float32)
    return q, r, k


def test_plan_replays_match_search_l2(gts):
    import torch

    d = synth.gaussian_mixture(311, 30000, 64, 25, -5.0, 5.0, 1.0, 600, 600)
    X = d["objects"]
    pool = np.concatenate([d["range_queries"], d["knn_queries"]])
    extra = synth.gaussian_mixture(312, 2000, 64, 25, -5.0, 5.0, 1.0)["objects"]
    nq = 333   # five query tiles and a ragged tail
    _say(f"plan L2 30000 x 64, {nq} queries, 4 replays")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=8, fanout=8, leaf_size=64, seed=7, cache_limit=5000)
    plan = gts.Plan(idx, nq, capacity=400 * nq)
    rng = np.random.default_rng(31)
    for rep in range(4):
        q, r, k = _inputs(rng, pool, nq, 4.5, 7.5, 40)
        _fill(plan, q, r, k)
        plan.launch()
        # eager work on the same stream between the launch and the read
        ref = idx.search(_dev(q), radius=r, k=k, result="device")
        torch.randn(1 << 20, device="cuda").sum().item()
        got, st = plan.result()
        assert st == 0, st
        assert int(got.offsets[-1]) == int(ref.offsets[-1])
        _same(got, ref)
        _say(f"replay {rep}: {int(ref.offsets[-1])} answers identical")
        if rep == 1:
            # the oracle on this replay (float64 brute force)
            lists = got.to_lists()
            objs = O.ObjectSet(vecs=X)
            rq, kq = np.nonzero(k == 0)[0][:40], np.nonzero(k > 0)[0][:40]
            for i in rq:
                check_range([lists[i]], O.range_bf(objs, O.ObjectSet(vecs=q[i:i + 1]), float(r[i])), X, q[i:i + 1],
                            float(r[i]))
            for i in kq:
                check_knn([lists[i]], O.knn_bf(objs, O.ObjectSet(vecs=q[i:i + 1]), int(k[i])), X, q[i:i + 1],
                          int(k[i]))
            _say("replay 1 matches the oracle on 80 queries")
    # updates: the plan records its graph again before the next launch
    new_ids = idx.insert(extra[:700])
    assert idx.delete(np.arange(0, 30000, 11)) > 0
    for step in ("after updates", "after rebuild"):
        q, r, k = _inputs(rng, pool, nq, 4.5, 7.5, 40)
        _fill(plan, q, r, k)
        plan.launch()
        got, st = plan.result()
        ref = idx.search(_dev(q), radius=r, k=k, result="device")
        assert st == 0, st
        _same(got, ref)
        _say(f"{step}: identical")
        if step == "after updates":
            idx.update_batch(extra[700:], delete_ids=new_ids[::3])
            assert idx.info()["rebuilds"] >= 1
    plan.close()
    idx.close()


@pytest.mark.parametrize("metric", ["L1", "COSINE"])
def test_plan_other_metrics(gts, metric):
    d = synth.gaussian_mixture(320, 12000, 48, 15, -4.0, 4.0, 1.0, 300, 300)
    X = d["objects"]
    pool = np.concatenate([d["range_queries"], d["knn_queries"]])
    m = gts.L1_F32 if metric == "L1" else gts.COSINE_F32
    # radii near the 0.1% quantile of each metric's distances
    l1, ang = metric == "L1", metric == "COSINE"
    D = O.pair_distances(O.ObjectSet(vecs=X[:3000], l1=l1, angular=ang),
                         O.ObjectSet(vecs=pool[:50], l1=l1, angular=ang))
    r0 = float(np.quantile(D, 0.001))
    nq = 200
    _say(f"plan {metric} 12000 x 48, {nq} queries, r ~ {r0:.4f}")
    idx = gts.Index(_dev(X), m, num_pivots=8, fanout=8, leaf_size=64, seed=4)
    plan = gts.Plan(idx, nq, capacity=300 * nq)
    rng = np.random.default_rng(32)
    for rep in range(3):
        q, r, k = _inputs(rng, pool, nq, 0.8 * r0, 1.2 * r0, 25)
        _fill(plan, q, r, k)
        plan.launch()
        ref = idx.search(_dev(q), radius=r, k=k, result="device")
        got, st = plan.result()
        assert st == 0, st
        _same(got, ref)
        _say(f"{metric} replay {rep}: {int(ref.offsets[-1])} answers identical")
    plan.close()
    idx.close()


def test_plan_status_flags(gts):
    d = synth.gaussian_mixture(330, 20000, 32, 10, -5.0, 5.0, 1.0, 200, 0)
    X, Q = d["objects"], d["range_queries"]
    nq = 130
    _say("plan status flags")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=8, fanout=8, leaf_size=64, seed=5)
    q = Q[:nq].copy()
    r = np.full(nq, 5.0, np.float32)
    k = np.zeros(nq, np.int32)
    k[::2] = 9
    ref = idx.search(_dev(q), radius=r, k=k, result="device")
    total = int(ref.offsets[-1])
    assert total > 10
    # answers beyond the capacity: flag 8, offsets[nq] the full count
    small = gts.Plan(idx, nq, capacity=total // 2)
    _fill(small, q, r, k)
    small.launch()
    got, st = small.result()
    assert st == gts.PLAN_ANSWERS
    assert int(got.offsets[-1]) == total
    assert np.array_equal(got.offsets.cpu().numpy(), ref.offsets.cpu().numpy())
    small.close()
    plan = gts.Plan(idx, nq, capacity=100 * nq)
    # a negative radius on a range query, then a negative k: flag 1
    for bad_r, bad_k in ((-1.0, 0), (5.0, -3)):
        r2, k2 = r.copy(), k.copy()
        r2[1], k2[1] = bad_r, bad_k
        _fill(plan, q, r2, k2)
        plan.launch()
        _, st = plan.result()
        assert st & gts.PLAN_BAD_INPUT, st
    # a NaN radius
    r2 = r.copy()
    r2[3] = np.nan
    _fill(plan, q, r2, k)
    plan.launch()
    assert plan.result()[1] & gts.PLAN_BAD_INPUT
    # a non-finite query value: flag 2
    q2 = q.copy()
    q2[5, 7] = np.inf
    _fill(plan, q2, r, k)
    plan.launch()
    assert plan.result()[1] == gts.PLAN_BAD_QUERY
    # good inputs again: status back to 0, answers as eager
    _fill(plan, q, r, k)
    plan.launch()
    got, st = plan.result()
    assert st == 0
    _same(got, ref)
    plan.close()
    # candidates beyond the plan's intermediate space: flag 4
    tight = gts.Plan(idx, nq, capacity=nq * 20000, mem_budget_bytes=24 << 20)
    _fill(tight, q, np.full(nq, 1e4, np.float32), np.zeros(nq, np.int32))
    tight.launch()
    assert tight.result()[1] & gts.PLAN_CANDIDATES
    tight.close()
    idx.close()


def test_plan_refuses_edit_index(gts):
    dd = synth.dna_families(340, 10, 20, 40, 60, 0.05, 4)
    chars, off = dd["objects"]
    idx = gts.Index((_dev(chars), _dev(off)), gts.EDIT_U8, num_pivots=4, fanout=4, seed=3)
    with pytest.raises(gts.GtsError) as e:
        gts.Plan(idx, 16, capacity=100)
    assert e.value.status == gts.ENOTSUP
    idx.close()
