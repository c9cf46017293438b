"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Every case prints its name before touching the GPU.  Inputs come from the
seeded generators; expected answers from oracle/ only.
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
RADII = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))
MODES = ("batched", "plain")


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


def _mode(g, name):
    return g.MODE_PLAIN if name == "plain" else g.MODE_BATCHED


@pytest.mark.parametrize("mode", MODES)
def test_l2_10k_d16(gts, mode):
    d = synth.make_workload("l2_10k_d16")
    X, RQ, KQ = d["objects"], d["range_queries"], d["knn_queries"]
    r = RADII["l2_10k_d16"]["radius_f32"]
    _say(f"l2_10k_d16 mode={mode}")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=5, fanout=8, leaf_size=64, seed=966001)
    Q = np.concatenate([RQ, KQ])
    k = np.array([0] * len(RQ) + [10] * len(KQ), np.int32)
    res = idx.search(_dev(Q), radius=np.full(len(Q), r, np.float32), k=k, mode=_mode(gts, mode)).to_lists()
    objs = O.ObjectSet(vecs=X)
    check_range(res[:100], O.range_bf(objs, O.ObjectSet(vecs=RQ), r), X, RQ, r)
    check_knn(res[100:], O.knn_bf(objs, O.ObjectSet(vecs=KQ), 10), X, KQ, 10)
    st = idx.stats()
    assert st["verified"] < len(Q) * len(X)          # the tree prunes
    idx.close()


@pytest.mark.parametrize("dim", [129, 200])
def test_l2_wide_rows(gts, dim):
    """Rows wider than the MFMA path (more than 128 floats) take the float32
    path in either mode, and its verification loops over the row."""
    d = synth.gaussian_mixture(70 + dim, 3000, dim, 5, -4.0, 4.0, 1.0, 30, 30)
    X, RQ, KQ = d["objects"], d["range_queries"], d["knn_queries"]
    objs = O.ObjectSet(vecs=X)
    # a radius that holds about 40 answers around the first range query
    r = float(O.knn_bf(objs, O.ObjectSet(vecs=RQ[:1]), 40)[0][1][-1])
    _say(f"l2 wide rows dim={dim} r={r}")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=6, fanout=4, leaf_size=64, seed=dim)
    Q = np.concatenate([RQ, KQ])
    k = np.array([0] * len(RQ) + [12] * len(KQ), np.int32)
    res = idx.search(_dev(Q), radius=np.full(len(Q), r, np.float32), k=k).to_lists()
    check_range(res[:30], O.range_bf(objs, O.ObjectSet(vecs=RQ), r), X, RQ, r)
    check_knn(res[30:], O.knn_bf(objs, O.ObjectSet(vecs=KQ), 12), X, KQ, 12)
    idx.close()


@pytest.mark.parametrize("kind", ["l2", "edit"])
def test_segments_beyond_the_lds_sort(gts, kind):
    """Queries whose candidate lists exceed what one workgroup sorts in LDS
    (thousands of answers each) take the global-memory sort."""
    _say(f"big segments {kind}")
    if kind == "l2":
        d = synth.gaussian_mixture(61, 12000, 8, 2, -1.0, 1.0, 1.0, 12, 12)
        X, RQ, KQ = d["objects"], d["range_queries"], d["knn_queries"]
        idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=4, fanout=4, leaf_size=64, seed=3)
        objs = O.ObjectSet(vecs=X)
        r = 3.0
        check_range(idx.range(_dev(RQ), r).to_lists(), O.range_bf(objs, O.ObjectSet(vecs=RQ), r), X, RQ, r)
        check_knn(idx.knn(_dev(KQ), 5000).to_lists(), O.knn_bf(objs, O.ObjectSet(vecs=KQ), 5000), X, KQ, 5000)
    else:
        items = synth.random_strings(62, 9000, 4, 9, b"AC")
        q = synth.random_strings(63, 10, 4, 9, b"AC")
        idx = gts.Index(items, gts.EDIT_U8, num_pivots=3, fanout=4, seed=4)
        objs, qs = O.ObjectSet(strings=items), O.ObjectSet(strings=q)
        check_exact(idx.range(q, 3.0, result="host").to_lists(), O.range_bf(objs, qs, 3.0))
        check_exact(idx.knn(q, 4000, result="host").to_lists(), O.knn_bf(objs, qs, 4000))
    assert max(len(a) for a, _ in idx.range(_dev(RQ) if kind == "l2" else q, 3.0, result="host").to_lists()) > 2048
    idx.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,dim", [(1, 3), (5, 3), (40, 3), (300, 33), (700, 2)])
def test_l2_tiny_exhaustive(gts, mode, n, dim):
    rng = np.random.default_rng(n * 7 + dim)
    base = rng.integers(-3, 4, size=(max(1, n // 3), dim)).astype(np.float32)
    X = base[rng.integers(0, base.shape[0], size=n)]             # exact duplicates
    Q = np.concatenate([X[: min(n, 6)], rng.integers(-3, 4, size=(6, dim)).astype(np.float32)])
    objs, qs = O.ObjectSet(vecs=X), O.ObjectSet(vecs=Q)
    _say(f"l2_tiny n={n} dim={dim} mode={mode}")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=3, fanout=2, leaf_size=4, seed=n)
    radii = np.unique(O.pair_distances(objs, qs).astype(np.float32))
    for r in list(radii[:: max(1, len(radii) // 6)]) + [0.0]:
        res = idx.range(_dev(Q), float(r), mode=_mode(gts, mode)).to_lists()
        check_range(res, O.range_bf(objs, qs, float(r)), X, Q, float(r))
    for k in sorted({1, 2, max(1, n // 2), n, n + 3}):
        res = idx.knn(_dev(Q), k, mode=_mode(gts, mode)).to_lists()
        check_knn(res, O.knn_bf(objs, qs, k), X, Q, k)
    idx.close()


@pytest.mark.parametrize("mode", MODES)
def test_l2_d128_several_tiles_ragged(gts, mode):
    # 20,000 x 128 from a 20-component mixture; 2 range + kNN query tiles and a
    # ragged third (150 queries); slabs of 256 rows with a ragged last slab
    d = synth.gaussian_mixture(777, 20_003, 128, 20, -5.0, 5.0, 1.0, 75, 75)
    X = d["objects"]
    Q = np.concatenate([d["range_queries"], d["knn_queries"]])
    objs = O.ObjectSet(vecs=X)
    D = O.pair_distances(objs, O.ObjectSet(vecs=d["range_queries"]))
    r = float(np.float32(np.sort(D.ravel())[int(0.002 * D.size)]))
    _say(f"l2_d128 n=20003 mode={mode} r={r}")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=16, fanout=16, leaf_size=256, seed=5)
    k = np.array([0] * 75 + [16] * 75, np.int32)
    res = idx.search(_dev(Q), radius=np.full(150, r, np.float32), k=k, mode=_mode(gts, mode)).to_lists()
    check_range(res[:75], O.range_bf(objs, O.ObjectSet(vecs=Q[:75]), r), X, Q[:75], r)
    check_knn(res[75:], O.knn_bf(objs, O.ObjectSet(vecs=Q[75:]), 16), X, Q[75:], 16)
    idx.close()


def test_knn_bound_small_incoherent_batches(gts):
    # 200,000 x 128 from a 100-component mixture, leaves of up to 256 rows;
    # batches of 8-48 kNN queries drawn from anywhere in the space (k 60-100),
    # so a 16-query block shares its MFMA window with unrelated queries.  The
    # bound must not take its k-th value from those queries' leaves: every
    # query keeps a small candidate set (a few per cent of the objects at
    # most), and the answers match the oracle.
    d = synth.gaussian_mixture(401, 200_000, 128, 100, -5.0, 5.0, 1.0, 2000, 0)
    X, pool = d["objects"], d["range_queries"]
    _say("kNN bound, small incoherent batches on 200000 x 128")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=16, fanout=16, leaf_size=256, seed=3)
    rng = np.random.default_rng(9)
    for nq in (8, 16, 48):
        for rep in range(6):
            q = pool[rng.choice(len(pool), nq, replace=False)]
            k = rng.integers(60, 101, nq).astype(np.int32)
            res = idx.search(_dev(q), k=k, result="device")
            worst = int(idx.stats()["max_query_candidates"])
            assert worst <= 5000, (nq, rep, worst)
        lists = res.to_lists()
        objs = O.ObjectSet(vecs=X)
        for i in range(min(nq, 8)):
            check_knn([lists[i]], O.knn_bf(objs, O.ObjectSet(vecs=q[i:i + 1]), int(k[i])), X, q[i:i + 1], int(k[i]))
        _say(f"nq={nq}: largest candidate set {worst}, answers match the oracle")
    idx.close()


@pytest.mark.parametrize("mode", MODES)
def test_edit_dna_families(gts, mode):
    d = synth.dna_families(31337, 60, 80, 64, 128, 0.05, 2)
    chars, off = d["objects"]
    qc, qo = d["queries"]
    nq = len(qo) - 1
    objs = O.ObjectSet(strings=(chars, off))
    _say(f"edit_dna n={len(off) - 1} nq={nq} mode={mode}")
    idx = gts.Index((_dev(chars), _dev(off)), gts.EDIT_U8, num_pivots=8, fanout=8, seed=3)
    for r in (0, 3, 8, 12):
        res = idx.range((_dev(qc), _dev(qo)), float(r), mode=_mode(gts, mode)).to_lists()
        check_exact(res, O.range_bf(objs, O.ObjectSet(strings=(qc, qo)), float(r)))
    for k in (1, 5, 40):
        res = idx.knn((_dev(qc), _dev(qo)), k, mode=_mode(gts, mode)).to_lists()
        check_exact(res, O.knn_bf(objs, O.ObjectSet(strings=(qc, qo)), k))
    idx.close()


def test_edit_edge_strings(gts):
    items = [b"", b"A", b"AC", b"ACGT" * 10, b"T" * 255, b"G" * 200, b"ACGTTGCA" * 16, b"CA"]
    chars, off = synth.strings_from_bytes(items * 5)
    q_items = [b"", b"A", b"T" * 250, b"ACGT" * 9, b"GGGG"]
    qc, qo = synth.strings_from_bytes(q_items)
    objs = O.ObjectSet(strings=(chars, off))
    qs = O.ObjectSet(strings=(qc, qo))
    _say("edit_edge_strings")
    idx = gts.Index((chars, off), gts.EDIT_U8, num_pivots=3, fanout=3, seed=1)
    for r in (0, 1, 5, 40, 255):
        check_exact(idx.range((qc, qo), float(r), result="host").to_lists(), O.range_bf(objs, qs, float(r)))
    for k in (1, 6, 40, 41):
        check_exact(idx.knn((qc, qo), k, result="host").to_lists(), O.knn_bf(objs, qs, k))
    idx.close()


def test_edit_alphabet_growth_and_foreign_bytes(gts):
    """Query bytes absent from the index match nothing; bytes first seen in
    an insert join the alphabet (cache scan, then the rebuilt tree)."""
    rng = np.random.default_rng(7)
    base = [bytes(rng.choice(list(b"ACGT"), int(rng.integers(0, 60))).tolist()) for _ in range(400)]
    extra = [b"ACGN" * 5, b"NNNN", b"Z" + b"ACGT" * 3, bytes(range(1, 60)), b"ACGTNACGTN"]
    q_items = [b"ACGN", b"NNNZ", b"\xff\xfeACG", b"ACGTACGT", bytes(range(1, 50)), b"", b"ZACGTACG"] + base[:70]
    qc, qo = synth.strings_from_bytes(q_items)
    qs = O.ObjectSet(strings=(qc, qo))
    _say("edit_alphabet")
    idx = gts.Index(synth.strings_from_bytes(base), gts.EDIT_U8, num_pivots=4, fanout=4, cache_limit=6, seed=3)
    new_ids = idx.insert(synth.strings_from_bytes(extra))           # stays in the cache list
    assert list(new_ids) == list(range(400, 405))
    for step in ("cache", "rebuilt"):
        items = base + extra
        objs = O.ObjectSet(strings=synth.strings_from_bytes(items))
        for mode in MODES:
            for r in (0, 2, 6, 20):
                check_exact(idx.range((qc, qo), float(r), mode=_mode(gts, mode), result="host").to_lists(),
                            O.range_bf(objs, qs, float(r)))
            for k in (1, 5, 30):
                check_exact(idx.knn((qc, qo), k, mode=_mode(gts, mode), result="host").to_lists(),
                            O.knn_bf(objs, qs, k))
        if step == "cache":
            more = [b"NNZZ", b"ACGTZ" * 4]
            idx.insert(synth.strings_from_bytes(more))                 # past the limit: rebuild
            extra = extra + more
            assert idx.info()["rebuilds"] == 1
    idx.close()


def test_edit_full_byte_alphabet(gts):
    """Every byte value occurs: the widest match tables (257 rows)."""
    rng = np.random.default_rng(8)
    items = [bytes(rng.integers(0, 256, int(rng.integers(0, 120))).astype(np.uint8).tolist()) for _ in range(600)]
    items += [bytes(range(0, 255)), bytes(range(1, 256))]
    q_items = [bytes(bytearray(s[:100])[::-1]) for s in items[:40]] + [items[5], items[-1], b"\x00" * 10]
    chars, off = synth.strings_from_bytes(items)
    qc, qo = synth.strings_from_bytes(q_items)
    objs, qs = O.ObjectSet(strings=(chars, off)), O.ObjectSet(strings=(qc, qo))
    _say("edit_full_alphabet")
    idx = gts.Index((_dev(chars), _dev(off)), gts.EDIT_U8, num_pivots=5, fanout=4, seed=5)
    for mode in MODES:
        for r in (0, 3, 60, 130):
            check_exact(idx.range((_dev(qc), _dev(qo)), float(r), mode=_mode(gts, mode)).to_lists(),
                        O.range_bf(objs, qs, float(r)))
        for k in (1, 7):
            check_exact(idx.knn((_dev(qc), _dev(qo)), k, mode=_mode(gts, mode)).to_lists(), O.knn_bf(objs, qs, k))
    idx.close()


def _live_set_l2(X, ids_all, live_ids):
    rows = {int(i): r for r, i in enumerate(ids_all)}
    sel = [rows[i] for i in sorted(live_ids)]
    return X[sel], np.array(sorted(live_ids), np.int64)


@pytest.mark.parametrize("cache_limit", [10_000, 50])
def test_l2_streamed_updates(gts, cache_limit):
    d = synth.gaussian_mixture(99, 4000, 20, 8, -6.0, 6.0, 1.0, 60, 60)
    X0 = d["objects"]
    extra = synth.gaussian_mixture(100, 300, 20, 8, -6.0, 6.0, 1.0)["objects"]
    _say(f"l2_updates cache_limit={cache_limit}")
    idx = gts.Index(_dev(X0), gts.L2_F32, num_pivots=8, fanout=4, leaf_size=32, cache_limit=cache_limit, seed=2)
    new_ids = idx.insert(_dev(extra))
    assert list(new_ids) == list(range(4000, 4300))
    rng = np.random.default_rng(1)
    dele = np.concatenate([rng.choice(4000, 250, replace=False), new_ids[rng.choice(300, 40, replace=False)]])
    assert idx.delete(dele) == len(dele)
    assert idx.delete(dele[:10]) == 0                     # already deleted
    assert idx.delete([10**6]) == 0                       # unknown id
    allX = np.concatenate([X0, extra])
    ids_all = np.arange(4300)
    live = set(range(4300)) - set(dele.tolist())
    Xl, idl = _live_set_l2(allX, ids_all, live)
    info = idx.info()
    assert info["n_live"] == len(live)
    if cache_limit < 300:
        assert info["rebuilds"] >= 1
    objs = O.ObjectSet(vecs=Xl, ids=idl)
    Q = np.concatenate([d["range_queries"], d["knn_queries"]])
    id_to_row = {int(i): int(i) for i in ids_all}
    for mode in MODES:
        res = idx.search(_dev(Q), radius=np.full(120, 3.0, np.float32), k=np.array([0] * 60 + [12] * 60, np.int32),
                         mode=_mode(gts, mode)).to_lists()
        check_range(res[:60], O.range_bf(objs, O.ObjectSet(vecs=Q[:60]), 3.0), allX, Q[:60], 3.0, id_to_row)
        check_knn(res[60:], O.knn_bf(objs, O.ObjectSet(vecs=Q[60:]), 12), allX, Q[60:], 12, id_to_row)
    idx.close()


def test_edit_streamed_updates(gts):
    d = synth.dna_families(7, 30, 40, 40, 80, 0.05, 2)
    chars, off = d["objects"]
    n0 = len(off) - 1
    e = synth.dna_families(8, 10, 10, 40, 80, 0.05)
    ec, eo = e["objects"]
    qc, qo = d["queries"]
    _say("edit_updates")
    idx = gts.Index((chars, off), gts.EDIT_U8, num_pivots=6, fanout=4, cache_limit=1000, seed=4)
    new_ids = idx.insert((ec, eo))
    dele = np.concatenate([np.arange(0, n0, 7), new_ids[::3]])
    idx.delete(dele)
    items = [chars[off[i]:off[i + 1]].tobytes() for i in range(n0)] + \
            [ec[eo[i]:eo[i + 1]].tobytes() for i in range(len(eo) - 1)]
    live = sorted(set(range(len(items))) - set(dele.tolist()))
    lc, lo = synth.strings_from_bytes([items[i] for i in live])
    objs = O.ObjectSet(strings=(lc, lo), ids=np.array(live, np.int64))
    qs = O.ObjectSet(strings=(qc, qo))
    for mode in MODES:
        check_exact(idx.range((qc, qo), 6.0, mode=_mode(gts, mode), result="host").to_lists(),
                    O.range_bf(objs, qs, 6.0))
        check_exact(idx.knn((qc, qo), 9, mode=_mode(gts, mode), result="host").to_lists(), O.knn_bf(objs, qs, 9))
    idx.close()


def test_two_stage_budget_gives_same_answers(gts):
    d = synth.gaussian_mixture(55, 6000, 32, 10, -5.0, 5.0, 1.0, 200, 200)
    X = d["objects"]
    Q = np.concatenate([d["range_queries"], d["knn_queries"]])
    _say("two_stage_budget")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=8, fanout=8, leaf_size=64, seed=1)
    k = np.array([0] * 200 + [20] * 200, np.int32)
    radius = np.full(400, 5.0, np.float32)
    big = idx.search(_dev(Q), radius=radius, k=k).to_lists()
    assert idx.stats()["groups"] == 1
    cands = idx.stats()["candidates"]
    # a budget for about a third of the batch's candidates: several groups run
    # one after another, each of whole 64-query tiles
    small = idx.search(_dev(Q), radius=radius, k=k, mem_budget_bytes=40 * (cands // 3)).to_lists()
    st = idx.stats()
    assert st["groups"] > 1
    # the groups are sized from the first attempt's counts, not by halving
    # until they fit: few overflowing attempts
    assert 1 <= st["group_retries"] <= 3, st
    for (a, b), (c, e) in zip(big, small):
        assert np.array_equal(a, c) and np.array_equal(b, e)
    objs = O.ObjectSet(vecs=X)
    check_range(small[:200], O.range_bf(objs, O.ObjectSet(vecs=Q[:200]), 5.0), X, Q[:200], 5.0)
    check_knn(small[200:], O.knn_bf(objs, O.ObjectSet(vecs=Q[200:]), 20), X, Q[200:], 20)
    idx.close()


def test_empty_batch_and_errors(gts):
    X = np.random.default_rng(0).standard_normal((100, 8)).astype(np.float32)
    _say("empty_and_errors")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=4, fanout=4)
    res = idx.range(_dev(np.zeros((0, 8), np.float32)), 1.0)
    assert len(res) == 0 and res.ids.numel() == 0
    with pytest.raises(gts.GtsError):
        idx.range(_dev(np.zeros((3, 7), np.float32)), 1.0)        # wrong dimension
    with pytest.raises(gts.GtsError):
        idx.range(_dev(np.zeros((3, 8), np.float32)), -1.0)       # negative radius
    with pytest.raises(gts.GtsError):
        idx.knn(_dev(np.zeros((3, 8), np.float32)), 0)            # k < 1
    with pytest.raises(gts.GtsError):
        gts.Index(_dev(X), gts.L2_F32, num_pivots=0, fanout=4)
    idx.close()


def test_candidate_count_beyond_32_bits(gts):
    """4,096 range queries whose radius admits every one of 2^20 objects make
    exactly 2^32 candidate reservations in the first group: a 32-bit count
    would wrap to 0 and pass the budget check with empty answers.  The
    64-bit count sees the overflow, the batch splits down to 64-query tiles,
    and a budget too small for one tile's candidates is an ENOMEM error."""
    n, dim, nq = 1 << 20, 16, 4096
    rng = np.random.default_rng(32)
    X = rng.uniform(-1.0, 1.0, size=(n, dim)).astype(np.float32)
    Q = rng.uniform(-1.0, 1.0, size=(nq, dim)).astype(np.float32)
    _say("candidate count beyond 32 bits")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=4, fanout=16, leaf_size=256, seed=3)
    with pytest.raises(gts.GtsError) as e:
        idx.range(_dev(Q), 1.0e4, mem_budget_bytes=256 << 20)
    assert e.value.status == gts.ENOMEM
    # the same radius on a few queries fits and returns every object
    res = idx.range(_dev(Q[:3]), 1.0e4).to_lists()
    assert all(len(ids) == n for ids, _ in res)
    idx.close()


def test_edit_two_stage_budget_gives_same_answers(gts):
    d = synth.dna_families(77, 60, 150, 60, 100, 0.05, 6)
    chars, off = d["objects"]
    qc, qo = d["queries"]
    nq = len(qo) - 1
    _say(f"edit two_stage_budget nq={nq}")
    idx = gts.Index((_dev(chars), _dev(off)), gts.EDIT_U8, num_pivots=6, fanout=6, seed=5)
    k = np.array([0, 5] * (nq // 2) + [0] * (nq % 2), np.int32)
    radius = np.full(nq, 7.0, np.float32)
    Qd = (_dev(qc), _dev(qo))
    big = idx.search(Qd, radius=radius, k=k).to_lists()
    assert idx.stats()["groups"] == 1
    cands = idx.stats()["candidates"]
    small = idx.search(Qd, radius=radius, k=k, mem_budget_bytes=40 * max(cands // 4, 1)).to_lists()
    assert idx.stats()["groups"] > 1
    idx.close()
    for (a, b), (c, e) in zip(big, small):
        assert np.array_equal(a, c) and np.array_equal(b, e)
    objs = O.ObjectSet(strings=(chars, off))
    for q in range(nq):
        qs = O.ObjectSet(strings=(qc[qo[q]:qo[q + 1]], np.array([0, qo[q + 1] - qo[q]], np.int64)))
        ref = O.knn_bf(objs, qs, 5)[0] if k[q] else O.range_bf(objs, qs, 7.0)[0]
        check_exact([small[q]], [ref])


def test_l2_planted_boundary_and_duplicates(gts):
    """Objects planted at float64 distance r * (1 + s) from each query for
    s in [-1e-6, 1e-6] (the bf16 estimates' error is far larger than those
    gaps), exact copies of the queries and duplicated objects: the bf16
    selection, the float32 selection and the plain form return identical
    answers, the oracle agrees within its tolerance, and no rechecked
    candidate left its bf16 interval."""
    base = synth.gaussian_mixture(91, 20000, 64, 20, -5.0, 5.0, 1.0, 64, 0)
    X0, Q = base["objects"], base["range_queries"]
    rng = np.random.default_rng(92)
    r = 6.0
    planted = []
    for q in Q.astype(np.float64):
        for s in (-1e-6, -3e-7, -1e-7, 0.0, 1e-7, 3e-7, 1e-6):
            for _ in range(3):
                u = rng.standard_normal(64)
                u /= np.linalg.norm(u)
                planted.append(q + r * (1.0 + s) * u)
        planted.append(q)                       # distance 0
    P = np.asarray(planted).astype(np.float32)
    X = np.concatenate([X0, P, P[:200], X0[:300]]).astype(np.float32)   # duplicates
    _say(f"planted boundary n={len(X)}")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=8, fanout=8, leaf_size=64, seed=9)
    Qd = _dev(np.concatenate([Q, Q]))
    k = np.array([0] * len(Q) + [45] * len(Q), np.int32)
    radius = np.full(2 * len(Q), r, np.float32)
    a = idx.search(Qd, radius=radius, k=k, flags=gts.QF_CHECK_BOUND).to_lists()
    st = idx.stats()
    assert st["bound_violations"] == 0 and st["verified"] > 0
    assert np.array_equal(np.concatenate([x[0] for x in a]),
                          np.concatenate([x[0] for x in idx.search(Qd, radius=radius, k=k).to_lists()]))
    b = idx.search(Qd, radius=radius, k=k, precision=gts.FP32).to_lists()
    c = idx.search(Qd, radius=radius, k=k, mode=gts.MODE_PLAIN).to_lists()
    idx.close()
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
        assert np.array_equal(x[0], z[0]) and np.array_equal(x[1], z[1])
    objs = O.ObjectSet(vecs=X)
    check_range(a[:len(Q)], O.range_bf(objs, O.ObjectSet(vecs=Q), r), X, Q, r)
    check_knn(a[len(Q):], O.knn_bf(objs, O.ObjectSet(vecs=Q), 45), X, Q, 45)


@pytest.mark.parametrize("mode", MODES)
def test_l2_precision_fp32_matches_oracle(gts, mode):
    d = synth.gaussian_mixture(95, 8000, 48, 12, -5.0, 5.0, 1.0, 150, 150)
    X = d["objects"]
    Q = np.concatenate([d["range_queries"], d["knn_queries"]])
    _say(f"precision fp32 mode={mode}")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=8, fanout=8, leaf_size=64, seed=2, precision=gts.FP32)
    k = np.array([0] * 150 + [17] * 150, np.int32)
    res = idx.search(_dev(Q), radius=np.full(300, 5.5, np.float32), k=k, mode=_mode(gts, mode)).to_lists()
    idx.close()
    objs = O.ObjectSet(vecs=X)
    check_range(res[:150], O.range_bf(objs, O.ObjectSet(vecs=Q[:150]), 5.5), X, Q[:150], 5.5)
    check_knn(res[150:], O.knn_bf(objs, O.ObjectSet(vecs=Q[150:]), 17), X, Q[150:], 17)


@pytest.mark.parametrize("metric", ["l2", "edit"])
def test_batch_update_rebuilds_and_matches_oracle(gts, metric):
    """The batch update of Sec. 4.4: 10% of the objects deleted and inserted
    back (fresh ids) in one call, with streamed inserts already waiting in
    the cache list; the index is rebuilt and answers match the oracle over
    the live set."""
    rng = np.random.default_rng(60)
    if metric == "l2":
        d = synth.gaussian_mixture(61, 6000, 24, 10, -5.0, 5.0, 1.0, 80, 80)
        X = d["objects"]
        Q = np.concatenate([d["range_queries"], d["knn_queries"]])
        idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=6, fanout=6, leaf_size=48, seed=2, cache_limit=100000)
        objs_all = [X[i] for i in range(len(X))]
    else:
        dd = synth.dna_families(62, 30, 100, 50, 90, 0.05, 3)
        chars, off = dd["objects"]
        qc, qo = dd["queries"]
        idx = gts.Index((_dev(chars), _dev(off)), gts.EDIT_U8, num_pivots=5, fanout=5, seed=3, cache_limit=100000)
        objs_all = [chars[off[i]:off[i + 1]].tobytes() for i in range(len(off) - 1)]
    n0 = len(objs_all)
    _say(f"batch update {metric} n={n0}")
    # a few streamed inserts first (they sit in the cache list)
    pre = objs_all[:25]
    pre_ids = idx.insert(np.stack(pre) if metric == "l2" else synth.strings_from_bytes(pre))
    assert idx.info()["n_cache"] == 25
    gone = rng.choice(n0, n0 // 10, replace=False)
    back = [objs_all[i] for i in gone]
    new_ids, nd = idx.update_batch(np.stack(back) if metric == "l2" else synth.strings_from_bytes(back), gone)
    assert nd == len(gone) and len(new_ids) == len(gone)
    info = idx.info()
    assert info["n_cache"] == 0 and info["rebuilds"] == 1 and info["n_live"] == n0 + 25
    live = {i: objs_all[i] for i in range(n0) if i not in set(gone.tolist())}
    live.update({int(i): o for i, o in zip(pre_ids, pre)})
    live.update({int(i): o for i, o in zip(new_ids, back)})
    ids = np.array(sorted(live), np.int64)
    if metric == "l2":
        Xl = np.stack([live[int(i)] for i in ids]).astype(np.float32)
        oset = O.ObjectSet(vecs=Xl, ids=ids)
        r = 5.0
        k = np.array([0] * 80 + [14] * 80, np.int32)
        res = idx.search(_dev(Q), radius=np.full(160, r, np.float32), k=k).to_lists()
        row = {int(i): j for j, i in enumerate(ids)}
        check_range(res[:80], O.range_bf(oset, O.ObjectSet(vecs=Q[:80]), r), Xl, Q[:80], r, id_to_row=row)
        check_knn(res[80:], O.knn_bf(oset, O.ObjectSet(vecs=Q[80:]), 14), Xl, Q[80:], 14, id_to_row=row)
    else:
        sc, so = synth.strings_from_bytes([live[int(i)] for i in ids])
        oset = O.ObjectSet(strings=(sc, so), ids=ids)
        nq = len(qo) - 1
        k = np.array([0, 4] * (nq // 2) + [0] * (nq % 2), np.int32)
        res = idx.search((_dev(qc), _dev(qo)), radius=np.full(nq, 6.0, np.float32), k=k).to_lists()
        for q in range(nq):
            qs = O.ObjectSet(strings=(qc[qo[q]:qo[q + 1]], np.array([0, qo[q + 1] - qo[q]], np.int64)))
            ref = O.knn_bf(oset, qs, 4)[0] if k[q] else O.range_bf(oset, qs, 6.0)[0]
            check_exact([res[q]], [ref])
    idx.close()


def test_no_prune_control_gives_same_answers(gts):
    """GTS_QF_NO_PRUNE (every (leaf, query) pair kept, the dense control)
    returns the answers of the pruned search; it computes more tiles."""
    d = synth.gaussian_mixture(71, 20000, 96, 20, -5.0, 5.0, 1.0, 200, 200)
    X = d["objects"]
    Q = np.concatenate([d["range_queries"], d["knn_queries"]])
    _say("no-prune control")
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=8, fanout=8, leaf_size=64, seed=4)
    k = np.array([0] * 200 + [10] * 200, np.int32)
    radius = np.full(400, 9.0, np.float32)
    a = idx.search(_dev(Q), radius=radius, k=k).to_lists()
    tiles_pruned = idx.stats()["tile_pairs"]
    b = idx.search(_dev(Q), radius=radius, k=k, flags=gts.QF_NO_PRUNE).to_lists()
    tiles_dense = idx.stats()["tile_pairs"]
    idx.close()
    assert tiles_dense > tiles_pruned
    for x, y in zip(a, b):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


def test_choose_fanout_from_a_sample(gts):
    d = synth.make_workload("l2_10k_d16")
    _say("choose fanout")
    best, costs = gts.choose_fanout(d["objects"], gts.L2_F32, 2.0, concurrency=1e5)
    assert 2 <= best <= 64 and np.all(np.isfinite(costs))
    assert costs[best - 2] == costs.min()
    dd = synth.dna_families(81, 10, 20, 40, 60, 0.05, 0)
    best_e, costs_e = gts.choose_fanout(dd["objects"], gts.EDIT_U8, 6.0, concurrency=1e5)
    assert 2 <= best_e <= 64 and costs_e[best_e - 2] == costs_e.min()
