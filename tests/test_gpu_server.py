"""The continuous-batching server against the oracle.

A scripted stream of range / kNN requests and insert / delete batches goes to
an L2 index and an edit-distance index served together.  Every query request
must equal the oracle's answer over the live set at its submission (its
admission epoch), and requests that were batched with others must give the
same answers as the same request alone on the index.
"""
import numpy as np
import pytest

import oracle as O
from paper_2404_00966_amd import synth
from tests.parity import check_exact, check_knn, check_range

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gts():
    import torch

    from paper_2404_00966_amd import gts as g

    assert torch.cuda.is_available()
    g.library()
    return g


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _strings(chars, off):
    return [chars[off[i]:off[i + 1]].tobytes() for i in range(len(off) - 1)]


def _drain(srv, n):
    out = {}
    while len(out) < n:
        for c in srv.poll(64, wait_ms=2000):
            out[c["ticket"]] = c
    return out


def test_server_stream_matches_oracle_and_alone(gts):
    d = synth.gaussian_mixture(77, 3000, 24, 6, -6.0, 6.0, 1.0, 60, 60)
    X0, RQ, KQ = d["objects"], d["range_queries"], d["knn_queries"]
    extra = synth.gaussian_mixture(78, 400, 24, 6, -6.0, 6.0, 1.0)["objects"]
    allX = np.concatenate([X0, extra])
    dn = synth.dna_families(5, 20, 40, 40, 80, 0.05, 3)
    dc, do = dn["objects"]
    qs_e = _strings(*dn["queries"])
    ex = synth.dna_families(6, 10, 10, 40, 80, 0.05)
    allS = _strings(dc, do) + _strings(*ex["objects"])
    n0_e = len(do) - 1
    _say("server stream")
    l2 = gts.Index(X0, gts.L2_F32, num_pivots=6, fanout=4, leaf_size=32, cache_limit=150, seed=1)
    ed = gts.Index((dc, do), gts.EDIT_U8, num_pivots=5, fanout=4, cache_limit=60, seed=2)
    srv = gts.Server([l2, ed], lanes_per_index=2, max_batch_queries=48)
    rng = np.random.default_rng(3)
    live = [set(range(3000)), set(range(n0_e))]
    next_id = [3000, n0_e]
    used = [0, 0]                                  # rows of `extra` / extra strings inserted so far
    meta = {}
    for step in range(160):
        u = rng.random()
        if u < 0.12:                               # update
            ix = int(rng.integers(0, 2))
            if rng.random() < 0.5 and used[ix] < (400 if ix == 0 else 100):
                m = int(rng.integers(1, 30))
                m = min(m, (400 if ix == 0 else 100) - used[ix])
                if ix == 0:
                    objs = extra[used[0]:used[0] + m]
                else:
                    objs = synth.strings_from_bytes(allS[n0_e + used[1]:n0_e + used[1] + m])
                used[ix] += m
                ids = list(range(next_id[ix], next_id[ix] + m))
                next_id[ix] += m
                live[ix] |= set(ids)
                t = srv.submit(("insert", ix, objs))
                meta[t] = ("insert", ix, ids)
            else:
                pool = sorted(live[ix])
                m = int(rng.integers(1, 40))
                dele = rng.choice(pool, size=min(m, len(pool)), replace=False).tolist() + [10 ** 6]
                expect = len(set(dele) & live[ix])
                live[ix] -= set(dele)
                t = srv.submit(("delete", ix, np.array(dele, np.int64)))
                meta[t] = ("delete", ix, expect, dele)
        else:
            ix = 0 if u < 0.72 else 1
            m = int(rng.integers(1, 9))
            snap = np.array(sorted(live[ix]), np.int64)
            if ix == 0:
                rows = rng.choice(60, size=m, replace=False)
                if rng.random() < 0.5:
                    r = float(rng.choice([2.0, 3.5, 5.0]))
                    t = srv.submit(("range", 0, RQ[rows], r))
                    meta[t] = ("range", 0, RQ[rows], r, snap)
                else:
                    k = int(rng.integers(1, 40))
                    t = srv.submit(("knn", 0, KQ[rows], k))
                    meta[t] = ("knn", 0, KQ[rows], k, snap)
            else:
                rows = rng.choice(len(qs_e), size=m, replace=False)
                q = synth.strings_from_bytes([qs_e[i] for i in rows])
                if rng.random() < 0.5:
                    r = float(rng.integers(0, 12))
                    t = srv.submit(("range", 1, q, r))
                    meta[t] = ("range", 1, q, r, snap)
                else:
                    k = int(rng.integers(1, 30))
                    t = srv.submit(("knn", 1, q, k))
                    meta[t] = ("knn", 1, q, k, snap)
    srv.flush()
    comps = _drain(srv, len(meta))
    st = srv.stats()
    assert st["completed"] == len(meta) and st["failed"] == 0
    batches = {}
    for t, c in comps.items():
        assert c["status"] == 0, c["error"]
        if c["batch"] >= 0:
            batches.setdefault(c["batch"], []).append(t)
    assert any(len(v) > 1 for v in batches.values()), "no batch admitted more than one request"
    for t, m in meta.items():
        c = comps[t]
        if m[0] == "insert":
            assert list(c["new_ids"]) == m[2]
            continue
        if m[0] == "delete":
            assert c["count"] == m[2]
            continue
        kind, ix, q, par, snap = m
        if ix == 0:
            objs = O.ObjectSet(vecs=allX[snap], ids=snap)
            qs = O.ObjectSet(vecs=q)
            if kind == "range":
                check_range(c["answers"], O.range_bf(objs, qs, par), allX, q, par)
            else:
                check_knn(c["answers"], O.knn_bf(objs, qs, par), allX, q, par)
        else:
            objs = O.ObjectSet(strings=synth.strings_from_bytes([allS[i] for i in snap]), ids=snap)
            qs = O.ObjectSet(strings=q)
            ref = O.range_bf(objs, qs, par) if kind == "range" else O.knn_bf(objs, qs, par)
            try:
                check_exact(c["answers"], ref)
            except AssertionError as e:
                # the updates of this index around the request, and its batch
                hist = [(u, meta[u][0], meta[u][2] if meta[u][0] == "insert" else meta[u][3])
                        for u in sorted(meta) if meta[u][0] in ("insert", "delete") and meta[u][1] == ix]
                mates = sorted(u for u, cc in comps.items() if cc["batch"] == c["batch"])
                raise AssertionError(f"ticket {t} ({kind}, {par}) batch {c['batch']} with {mates}; "
                                     f"updates {hist}: {e}") from None
    # alone vs in the mix: requests submitted after the last update of their
    # index see the final state; rerun them alone and compare bit for bit
    last_update = {0: 0, 1: 0}
    for t, m in meta.items():
        if m[0] in ("insert", "delete"):
            last_update[m[1]] = max(last_update[m[1]], t)
    srv.close()
    checked = 0
    for t, m in meta.items():
        if m[0] in ("range", "knn") and t > last_update[m[1]]:
            kind, ix, q, par, _ = m
            idx = l2 if ix == 0 else ed
            alone = idx.range(q, par, result="host") if kind == "range" else idx.knn(q, par, result="host")
            for (a, b), (e, f) in zip(comps[t]["answers"], alone.to_lists()):
                assert np.array_equal(a, e) and np.array_equal(b, f)
            checked += 1
    assert checked > 0
    l2.close()
    ed.close()


def test_server_rejects_bad_requests(gts):
    d = synth.gaussian_mixture(79, 500, 8, 3, -5.0, 5.0, 1.0, 4, 4)
    idx = gts.Index(d["objects"], gts.L2_F32, num_pivots=3, fanout=4, leaf_size=16, seed=1)
    srv = gts.Server([idx])
    _say("server errors")
    with pytest.raises(gts.GtsError):
        srv.submit(("knn", 0, d["knn_queries"], 0))
    with pytest.raises(gts.GtsError):
        srv.submit(("range", 0, d["range_queries"], -1.0))
    with pytest.raises(gts.GtsError):
        srv.submit(("range", 3, d["range_queries"], 1.0))
    with pytest.raises(gts.GtsError):
        srv.submit(("knn", 0, np.zeros((2, 5), np.float32), 3))
    t = srv.submit(("knn", 0, d["knn_queries"], 3))
    srv.flush()
    c = srv.poll(8, wait_ms=0)
    assert len(c) == 1 and c[0]["ticket"] == t and c[0]["status"] == 0
    assert srv.stats()["submitted"] == 1
    srv.close()
    idx.close()
