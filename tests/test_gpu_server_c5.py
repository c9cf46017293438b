"""The serving mix at its full index sizes against the oracle.

An L2 index of 2,000,000 x 128 (100-component Gaussian mixture, 16 pivots,
fanout 16, leaves of 256) and an edit-distance index of 200,000 DNA strings
(400 families of 500 mutants, 8 pivots, fanout 8) are served together.  A
short open-loop trace at 50,000 requests/s mixes kNN (k uniform on 1..100),
range queries (selectivity log-uniform on [0.001%, 0.1%], radius from the
quantile table the oracle wrote) and update batches of 1..1,000 objects,
half inserts and half deletes, on either index.  The cache limits are low
enough that both indexes rebuild during the trace.

A seeded sample of the query requests is checked against the oracle's brute
force over the live set at the request's submission (its admission epoch):
the build objects and the inserted objects, less every id deleted by an
update submitted before it.
"""
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
from paper_2404_00966_amd import synth
from tests.parity import check_exact, check_knn, check_range

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _strings(chars, off):
    return [chars[off[i]:off[i + 1]].tobytes() for i in range(len(off) - 1)]


def test_server_c5_sizes_sampled_oracle():
    import torch

    from paper_2404_00966_amd import gts

    assert torch.cuda.is_available()
    radii = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))
    tl2, tdna = radii["serve_l2_2m_d128"], radii["serve_dna_200k"]
    sel_grid = np.log(np.asarray(tl2["selectivity"]))
    r_grid = np.asarray(tl2["radius_f32"])
    within = np.asarray(tdna["within_r"])
    _say("serving workloads 2M x 128 + 200k DNA")
    wl = synth.make_serving("serve_l2_2m_d128")
    wd = synth.make_serving("serve_dna_200k")
    n0 = [len(wl["objects"]), len(wd["objects"][1]) - 1]
    allX = np.concatenate([wl["objects"], wl["inserts"]])
    allS = _strings(*wd["objects"]) + _strings(*wd["inserts"])
    ql2 = wl["queries"]
    qs_dna = _strings(*wd["queries"])

    il2 = gts.Index(torch.from_numpy(wl["objects"]).cuda(), gts.L2_F32, num_pivots=wl["pivots"],
                    fanout=wl["fanout"], leaf_size=wl["leaf"], seed=wl["seed"], cache_limit=4000)
    oc, oo = wd["objects"]
    idna = gts.Index((torch.from_numpy(oc).cuda(), torch.from_numpy(oo).cuda()), gts.EDIT_U8,
                     num_pivots=wd["pivots"], fanout=wd["fanout"], seed=wd["seed"], cache_limit=4000)
    _say("indexes built")

    rng = np.random.default_rng(966008)
    alive = [np.ones(len(allX), bool), np.ones(len(allS), bool)]
    next_id = list(n0)
    del_log = [[], []]                 # deleted ids per index, in submission order
    reqs, meta = [], []
    n_req = 1500
    for i in range(n_req):
        ix = int(rng.integers(0, 2))
        u = rng.random()
        if u < 0.95:
            m = int(rng.integers(1, 5))
            if ix == 0:
                q = ql2[rng.choice(len(ql2), size=m, replace=False)]
            else:
                q = synth.strings_from_bytes([qs_dna[j] for j in rng.choice(len(qs_dna), size=m, replace=False)])
            if u < 0.70:
                par = int(rng.integers(1, 101))
                reqs.append(("knn", ix, q, par))
            else:
                s = float(np.exp(rng.uniform(np.log(1e-5), np.log(1e-3))))
                if ix == 0:
                    par = float(np.interp(np.log(s), sel_grid, r_grid))
                else:
                    ok = np.nonzero(within <= s)[0]
                    par = float(ok[-1]) if len(ok) else 0.0
                reqs.append(("range", ix, q, par))
            meta.append((reqs[-1][0], ix, q, par, None))
        else:
            m = int(rng.integers(1, 1001))
            if rng.random() < 0.5:
                m = min(m, len(alive[ix]) - next_id[ix])
                a, b = next_id[ix], next_id[ix] + m
                if ix == 0:
                    objs = allX[a:b]
                else:
                    objs = synth.strings_from_bytes(allS[a:b])
                next_id[ix] = b
                reqs.append(("insert", ix, objs))
                meta.append(("insert", ix, list(range(a, b)), None, None))
            else:
                cand = np.nonzero(alive[ix][:next_id[ix]])[0]
                ids = rng.choice(cand, size=min(m, len(cand)), replace=False)
                alive[ix][ids] = False
                del_log[ix].append(ids)
                reqs.append(("delete", ix, ids.astype(np.int64)))
                meta.append(("delete", ix, len(ids), None, None))
        if meta[-1][0] in ("knn", "range"):
            # the live set this request must see: everything inserted so far,
            # less everything deleted so far
            meta[-1] = meta[-1][:4] + ((next_id[ix], len(del_log[ix])),)
    kinds = [m[0] for m in meta]
    assert kinds.count("insert") > 10 and kinds.count("delete") > 10
    _say(f"trace of {n_req} requests at 50,000/s")
    srv = gts.Server([il2, idna], lanes_per_index=2)
    arrival = np.arange(n_req, dtype=np.float64) * (1e3 / 50_000.0)
    tickets = srv.replay(reqs, arrival)
    comps = {}
    while len(comps) < n_req:
        for c in srv.poll(256, wait_ms=2000):
            comps[c["ticket"]] = c
    srv.flush()
    st = srv.stats()
    srv.close()
    _say(f"trace drained: {st}")
    assert st["completed"] == n_req and st["failed"] == 0
    rebuilds = [il2.info()["rebuilds"], idna.info()["rebuilds"]]
    assert rebuilds[0] >= 1 and rebuilds[1] >= 1, rebuilds

    by_req = [comps[int(t)] for t in tickets]
    for c, m in zip(by_req, meta):
        assert c["status"] == 0, c["error"]
        if m[0] == "insert":
            assert list(c["new_ids"]) == m[2]
        elif m[0] == "delete":
            assert c["count"] == m[2]
    # a seeded sample of query requests per index, spread over the trace
    qpos = [[i for i, m in enumerate(meta) if m[0] in ("knn", "range") and m[1] == ix] for ix in (0, 1)]
    sample = sorted(rng.choice(qpos[0], size=10, replace=False).tolist() +
                    rng.choice(qpos[1], size=6, replace=False).tolist())

    def check(i):
        kind, ix, q, par, (nid, ndel) = meta[i]
        live = np.ones(nid, bool)
        for ids in del_log[ix][:ndel]:
            live[ids] = False
        snap = np.nonzero(live)[0]
        ans = by_req[i]["answers"]
        if ix == 0:
            objs = O.ObjectSet(vecs=allX[snap], ids=snap)
            qs = O.ObjectSet(vecs=q)
            if kind == "range":
                check_range(ans, O.range_bf(objs, qs, par), allX, q, par)
            else:
                check_knn(ans, O.knn_bf(objs, qs, par), allX, q, par)
        else:
            objs = O.ObjectSet(strings=synth.strings_from_bytes([allS[j] for j in snap]), ids=snap)
            qs = O.ObjectSet(strings=q)
            check_exact(ans, O.range_bf(objs, qs, par) if kind == "range" else O.knn_bf(objs, qs, par))
        return i

    _say(f"oracle on {len(sample)} sampled requests")
    with ThreadPoolExecutor(max_workers=8) as ex:
        for i in ex.map(check, sample):
            _say(f"request {i} ({meta[i][0]} on index {meta[i][1]}) matches the oracle")
    il2.close()
    idna.close()
