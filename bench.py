"""Benchmark: batched metric search on one MI355X.

Default workload (one step = one mixed batch through the whole search path):
  l2_1m_d128: 1,000,000 x 128 float32 vectors (100-component Gaussian
  mixture), 16 pivots, fanout 16, leaf 256; 10,000 kNN queries (k = 16) plus
  10,000 range queries at the 0.01% distance quantile, in one call.
Reported alongside (same JSON line, key "dna_500k"): 500,000 DNA strings
(1,000 families x 500 mutants), 8 pivots, fanout 8; 10,000 range queries
r = 8 per step.

Inputs are resident in HBM before timing; a step is gts_search on the whole
batch with answers left in device memory.  Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "queries/s oracle-exact: 1M×128 L2 kNN k=16, 500k DNA edit range r=8; p99 ms"
BF16_PEAK_TFLOPS = 2500.0       # MI355X dense bf16 MFMA
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_steps(fn, steps, warmup):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        per.append((time.perf_counter() - a) * 1e3)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return total, per


def pct(v, p):
    import numpy as np

    return float(np.percentile(np.asarray(v), p)) if v else None


def run_l2(args, gts, synth, torch, np):
    w = synth.WORKLOADS["l2_1m_d128"]
    radii = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))
    r = radii["l2_1m_d128"]["radius_f32"]
    t = time.perf_counter()
    d = synth.make_workload("l2_1m_d128", queries=args.queries)
    log(f"l2_1m_d128 generated in {time.perf_counter() - t:.1f}s")
    X = torch.from_numpy(d["objects"]).cuda()
    Q = torch.from_numpy(np.concatenate([d["knn_queries"], d["range_queries"]])).cuda()
    nk, nr = len(d["knn_queries"]), len(d["range_queries"])
    k = np.array([w["k"]] * nk + [0] * nr, np.int32)
    radius = np.full(nk + nr, r, np.float32)
    torch.cuda.synchronize()
    t = time.perf_counter()
    idx = gts.Index(X, gts.L2_F32, num_pivots=w["pivots"], fanout=w["fanout"], leaf_size=w["leaf"],
                    seed=w["seed"])
    build_s = time.perf_counter() - t
    log(f"index built in {build_s:.1f}s: {idx.info()}")
    # let the index's query context settle its tuned knob (untimed)
    tune_calls = 0
    for tune_calls in range(1, 17):
        idx.search(Q, radius=radius, k=k, result="device")
        if idx.stats()["tuning"] == 0:
            break
    log(f"tuning finished after {tune_calls} calls")
    total, per = timed_steps(lambda: idx.search(Q, radius=radius, k=k, result="device"), args.steps, args.warmup)
    nq = nk + nr
    qps = nq * args.steps / total
    # one more step with stage timing on, for the stage split and the roofline
    idx.set_timing(True)
    idx.search(Q, radius=radius, k=k, result="device")
    st = idx.stats()
    idx.set_timing(False)
    out = {"qps": qps, "ms_per_step": total * 1e3 / args.steps, "per_step_ms": per, "build_s": build_s,
           "stats": st, "nq": nq, "r": r, "k": w["k"], "n": d["n"], "dim": w["dim"],
           "tuned": {"bound_window": st["bound_window"], "tuning_calls": tune_calls}}
    if args.plain_queries > 0:
        sub = slice(0, args.plain_queries // 2)
        Qp = torch.cat([Q[:nk][sub], Q[nk:][sub]])
        kp = np.concatenate([k[:nk][sub], k[nk:][sub]])
        rp = np.concatenate([radius[:nk][sub], radius[nk:][sub]])
        tp, _ = timed_steps(lambda: idx.search(Qp, radius=rp, k=kp, mode=gts.MODE_PLAIN, result="device"), 1, 0)
        out["plain_qps"] = len(kp) / tp
        out["plain_queries"] = len(kp)
    idx.close()
    return out, d


def run_dna(args, gts, synth, torch, np):
    w = synth.WORKLOADS["dna_500k"]
    t = time.perf_counter()
    d = synth.make_workload("dna_500k", queries=args.queries)
    log(f"dna_500k generated in {time.perf_counter() - t:.1f}s")
    chars, off = d["objects"]
    qc, qo = d["queries"]
    nq = len(qo) - 1
    oc, oo = torch.from_numpy(chars).cuda(), torch.from_numpy(off).cuda()
    qct, qot = torch.from_numpy(qc).cuda(), torch.from_numpy(qo).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    idx = gts.Index((oc, oo), gts.EDIT_U8, num_pivots=w["pivots"], fanout=w["fanout"], seed=w["seed"])
    build_s = time.perf_counter() - t
    log(f"dna index built in {build_s:.1f}s: {idx.info()}")
    radius = np.full(nq, float(w["radius"]), np.float32)
    total, per = timed_steps(lambda: idx.search((qct, qot), radius=radius, result="device"), args.steps,
                             args.warmup)
    idx.set_timing(True)
    idx.search((qct, qot), radius=radius, result="device")
    st = idx.stats()
    idx.set_timing(False)
    out = {"qps": nq * args.steps / total, "ms_per_step": total * 1e3 / args.steps, "per_step_ms": per,
           "build_s": build_s, "stats": st, "nq": nq}
    if args.plain_queries > 0:
        m = min(nq, args.plain_queries)
        tp, _ = timed_steps(lambda: idx.search((qct, qot[: m + 1]), radius=radius[:m], mode=gts.MODE_PLAIN,
                                               result="device"), 1, 0)
        out["plain_qps"] = m / tp
        out["plain_queries"] = m
    idx.close()
    return out, d


def cpu_baseline(args, l2data, np):
    """The oracle's brute force (test infrastructure) on a bounded sample of
    the same workload, on the host cores."""
    import oracle as O

    radii = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))
    r = radii["l2_1m_d128"]["radius_f32"]
    m = args.cpu_queries // 2
    objs = O.ObjectSet(vecs=l2data["objects"])
    kq = O.ObjectSet(vecs=np.ascontiguousarray(l2data["knn_queries"][:m]))
    rq = O.ObjectSet(vecs=np.ascontiguousarray(l2data["range_queries"][:m]))
    t = time.perf_counter()
    O.knn_bf(objs, kq, 16)
    O.range_bf(objs, rq, r)
    el = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    return {"value": 2 * m / el, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"{m} kNN (k=16) + {m} range queries over all 1,000,000 x 128 objects, "
                      f"float64 brute force, {el:.1f}s"}


def run_serving(args, gts, synth, torch, np):
    """Serving mix: an L2 index (2M x 128) and a DNA index (200k strings)
    behind one continuous-batching server, driven by an open-loop Poisson
    trace: 70% kNN (k uniform 1..100), 25% range (selectivity log-uniform on
    [0.001%, 0.1%], radius from the oracle's quantile table), 5% update
    batches (1..N objects, insert or delete), each request on either index
    with equal probability.  Latency runs from submission to answers on the
    host.  A warm-up trace runs first on a separate server."""
    radii = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))
    tl2, tdna = radii["serve_l2_2m_d128"], radii["serve_dna_200k"]
    sel_grid = np.log(np.asarray(tl2["selectivity"]))
    r_grid = np.asarray(tl2["radius_f32"])
    within = np.asarray(tdna["within_r"])
    t = time.perf_counter()
    wl = synth.make_serving("serve_l2_2m_d128")
    wd = synth.make_serving("serve_dna_200k")
    log(f"serving workloads generated in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    il2 = gts.Index(torch.from_numpy(wl["objects"]).cuda(), gts.L2_F32, num_pivots=wl["pivots"],
                    fanout=wl["fanout"], leaf_size=wl["leaf"], seed=wl["seed"], cache_limit=args.serve_cache)
    oc, oo = wd["objects"]
    idna = gts.Index((torch.from_numpy(oc).cuda(), torch.from_numpy(oo).cuda()), gts.EDIT_U8,
                     num_pivots=wd["pivots"], fanout=wd["fanout"], seed=wd["seed"], cache_limit=args.serve_cache)
    build_s = time.perf_counter() - t
    log(f"serving indexes built in {build_s:.1f}s")
    rng = np.random.default_rng(966007)
    n_obj = [len(wl["objects"]), len(oo) - 1]
    # liveness by id (ids are assigned in submission order, updates apply in order)
    alive = [np.ones(2 * n_obj[0], bool), np.ones(2 * n_obj[1], bool)]
    next_id = list(n_obj)
    ins_used = [0, 0]
    ql2 = wl["queries"]
    qc, qo = wd["queries"]
    ic, io = wd["inserts"]

    def trace(seconds):
        n = int(rng.poisson(args.serve_rate * seconds))
        arr = np.cumsum(rng.exponential(1e3 / args.serve_rate, size=n))
        reqs = []
        for i in range(n):
            ix = int(rng.integers(0, 2))
            u = rng.random()
            if u < 0.70 or u < 0.95:
                if ix == 0:
                    j = int(rng.integers(0, len(ql2)))
                    q = ql2[j:j + 1]
                else:
                    j = int(rng.integers(0, len(qo) - 1))
                    q = (qc[qo[j]:qo[j + 1]], np.array([0, qo[j + 1] - qo[j]], np.int64))
                if u < 0.70:
                    reqs.append(("knn", ix, q, int(rng.integers(1, 101))))
                else:
                    s = float(np.exp(rng.uniform(np.log(1e-5), np.log(1e-3))))
                    if ix == 0:
                        r = float(np.interp(np.log(s), sel_grid, r_grid))
                    else:
                        ok = np.nonzero(within <= s)[0]
                        r = float(ok[-1]) if len(ok) else 0.0
                    reqs.append(("range", ix, q, r))
            else:
                m = int(rng.integers(1, args.serve_update_max + 1))
                if rng.random() < 0.5:
                    if ix == 0:
                        a = ins_used[0] % len(wl["inserts"])
                        b = min(a + m, len(wl["inserts"]))
                        objs = wl["inserts"][a:b]
                        cnt = b - a
                    else:
                        a = ins_used[1] % (len(io) - 1)
                        b = min(a + m, len(io) - 1)
                        objs = (ic[io[a]:io[b]], io[a:b + 1] - io[a])
                        cnt = b - a
                    ins_used[ix] += cnt
                    next_id[ix] += cnt
                    if next_id[ix] > len(alive[ix]):
                        alive[ix] = np.concatenate([alive[ix], np.ones(len(alive[ix]), bool)])
                    reqs.append(("insert", ix, objs))
                else:
                    ids = []
                    while len(ids) < m:
                        c = rng.integers(0, next_id[ix], size=2 * m)
                        c = np.unique(c[alive[ix][c]])
                        take = c[: m - len(ids)]
                        ids.extend(take.tolist())
                        alive[ix][take] = False
                    reqs.append(("delete", ix, np.array(ids[:m], np.int64)))
        return reqs, arr

    out = {}
    for phase, secs in (("warmup", args.serve_warmup_s), ("measured", args.serve_s)):
        reqs, arr = trace(secs)
        log(f"{phase}: {len(reqs)} requests over {secs}s")
        srv = gts.Server([il2, idna], lanes_per_index=args.serve_lanes, keep_results=False)
        t = time.perf_counter()
        srv.replay(reqs, arr)
        # drain, reporting the server's own completion count while it works
        last = time.perf_counter()
        while True:
            st = srv.stats()
            if st["completed"] + st["failed"] >= len(reqs):
                break
            time.sleep(0.05)
            if time.perf_counter() - last >= 10.0:
                log(f"{phase}: {st['completed']} of {len(reqs)} requests completed")
                last = time.perf_counter()
        srv.flush()
        wall = time.perf_counter() - t
        st = srv.stats()
        srv.close()
        kinds = {}
        for q in reqs:
            kinds[q[0]] = kinds.get(q[0], 0) + 1
        out[phase] = dict(st, wall_s=wall, requests=len(reqs), kinds=kinds,
                          offered_rate=len(reqs) / secs if secs else 0.0)
        log(f"{phase}: {st}")
    out["build_s"] = build_s
    out["rebuilds"] = [il2.info()["rebuilds"], idna.info()["rebuilds"]]
    il2.close()
    idna.close()
    return out


# HBM bytes per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE (each scaled by
# what the counters read for a plain 256 MiB device copy), per kernel, for
# the kernel source as profiled; None once the kernel has changed since.
TRAFFIC_BYTES = {"k_verify_l2": 687348230, "k_mfma_sweep": 623453968, "k_bound_near": 712193269}


def rooflines(st, dim):
    """Roofline points of the kernels behind the timed stages of one search
    call (stage times are HIP-event times on the index's stream; each stage
    is one kernel).  Algorithmic work per launch:
      k_mfma_sweep: every (query, object) pair of the computed (256-object
        slab, 16-query block) units, 2 * D flop each (D = dim rounded up to
        32);
      k_verify_l2: per candidate its 16-byte record and the 8 bytes of its
        norm and rounding error, per float32 recheck one object row (4 * dim
        bytes), per answer its 8-byte key;
      k_bound_near: one object row (4 * dim bytes) per distance of the kNN
        bound windows."""
    dk = (dim + 31) // 32 * 32
    out = {}
    ms = st["ms_stage"]["cands"]
    flops = 2.0 * dk * st["tile_pairs"] * 16 * 256
    a = flops / (ms * 1e-3) / 1e12 if ms > 0 else None
    out["k_mfma_sweep"] = {"bound": "mfma", "achieved": a, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": a / BF16_PEAK_TFLOPS if a else None, "traffic": TRAFFIC_BYTES["k_mfma_sweep"],
                           "work_per_launch": flops, "launch_ms": ms,
                           "work": "(256-object slab, 16-query block) units x 16 x 256 pairs x 2*Dk flop"}
    ms = st["ms_stage"]["verify"]
    byts = 24.0 * st["candidates"] + 4.0 * dim * st["verified"] + 8.0 * st["results"]
    a = byts / (ms * 1e-3) / 1e9 if ms > 0 else None
    out["k_verify_l2"] = {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": a / HBM_PEAK_GBS if a else None, "traffic": TRAFFIC_BYTES["k_verify_l2"],
                          "work_per_launch": byts, "launch_ms": ms,
                          "work": "24 B per candidate + 4*dim B per float32 recheck + 8 B per answer"}
    ms = st["ms_stage"]["bound"]
    byts = 4.0 * dim * st["bound_evals"]
    a = byts / (ms * 1e-3) / 1e9 if ms > 0 else None
    out["k_bound_near"] = {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": a / HBM_PEAK_GBS if a else None, "traffic": TRAFFIC_BYTES["k_bound_near"],
                           "work_per_launch": byts, "launch_ms": ms,
                           "work": "4*dim B per distance of the kNN bound windows"}
    return out


def calibrate_copy(torch):
    """A plain device copy of 256 MiB (one copy kernel), for scaling the
    profiler's HBM byte counters."""
    x = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    log("calibration copy: 268435456 bytes read, 268435456 written")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--queries", type=int, default=None, help="cap queries per kind (default: full)")
    ap.add_argument("--plain-queries", type=int, default=2000)
    ap.add_argument("--cpu-queries", type=int, default=1600)
    ap.add_argument("--skip-dna", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true", help="run one 256 MiB device copy first (profiling)")
    ap.add_argument("--serving", action="store_true", help="run the serving mix instead of the batch benchmark")
    ap.add_argument("--serve-rate", type=float, default=50000.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-s", type=float, default=4.0, help="measured trace length, s")
    ap.add_argument("--serve-warmup-s", type=float, default=1.0)
    ap.add_argument("--serve-update-max", type=int, default=1000)
    ap.add_argument("--serve-lanes", type=int, default=2)
    ap.add_argument("--serve-cache", type=int, default=1 << 20, help="cache list limit of the serving indexes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X and has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2404_00966_amd import gts, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    gts.library()
    if args.calibrate_copy:
        calibrate_copy(torch)
    if args.serving:
        sv = run_serving(args, gts, synth, torch, np)
        m = sv["measured"]
        qps = m["queries"] / (m["span_ms"] * 1e-3) if m["span_ms"] > 0 else 0.0
        line = {"metric": "queries/s, serving mix (2M x 128 L2 + 200k DNA, Poisson arrivals); p99 ms",
                "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": 1, "warmup": 1,
                "ms_per_step": m["span_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "bf16-mfma/f32 (L2), int32 (edit)", "data": "synthetic (seeded mixture / DNA families)",
                "config": {"workload": "serving_mix", "rate_per_s": args.serve_rate, "seconds": args.serve_s,
                           "update_max": args.serve_update_max, "lanes_per_index": args.serve_lanes,
                           "cache_limit": args.serve_cache},
                "p50_ms": m["p50_ms"], "p99_ms": m["p99_ms"], "serving": sv}
        print(json.dumps(line), flush=True)
        return
    l2, l2data = run_l2(args, gts, synth, torch, np)
    log(f"l2: {l2['qps']:.0f} q/s, {l2['ms_per_step']:.2f} ms/step, stages {l2['stats']['ms_stage']}")
    dna = None
    if not args.skip_dna:
        dna, _ = run_dna(args, gts, synth, torch, np)
        log(f"dna: {dna['qps']:.0f} q/s, {dna['ms_per_step']:.2f} ms/step, stages {dna['stats']['ms_stage']}")

    st = l2["stats"]
    roofs = rooflines(st, l2["dim"])
    # the roofline reported is the one of the kernel that takes longest
    dom = max(roofs, key=lambda name: roofs[name]["launch_ms"])
    roof = dict(roofs[dom], kernel=dom)
    cpu = None
    if args.cpu_queries > 0:
        log("cpu baseline (oracle brute force) ...")
        cpu = cpu_baseline(args, l2data, np)
    line = {
        "metric": METRIC,
        "value": l2["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": l2["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-mfma/f32",
        "data": "synthetic (seeded Gaussian mixture / DNA families)",
        "config": {"workload": "l2_1m_d128", "n": l2["n"], "dim": l2["dim"], "queries": l2["nq"],
                   "knn_k": l2["k"], "knn_queries": l2["nq"] // 2, "range_queries": l2["nq"] // 2,
                   "range_r": l2["r"], "pivots": 16, "fanout": 16, "leaf": 256},
        "p50_ms": pct(l2["per_step_ms"], 50),
        "p99_ms": pct(l2["per_step_ms"], 99),
        "latency_note": "batched: every query of a step completes with the step (makespan)",
        "stage_ms": l2["stats"]["ms_stage"],
        "counters": {k: l2["stats"][k] for k in ("node_tests", "tile_pairs", "candidates", "verified", "results",
                                                 "bound_evals")},
        "build_s": l2["build_s"],
        "tuned": l2["tuned"],
        "plain_qps": l2.get("plain_qps"),
        "plain_queries": l2.get("plain_queries"),
        "roofline": roof,
        "rooflines": roofs,
        "cpu_baseline": cpu,
    }
    if dna:
        line["dna_500k"] = {"queries_per_s": dna["qps"], "ms_per_step": dna["ms_per_step"],
                            "p50_ms": pct(dna["per_step_ms"], 50), "p99_ms": pct(dna["per_step_ms"], 99),
                            "queries": dna["nq"], "radius": 8, "build_s": dna["build_s"],
                            "stage_ms": dna["stats"]["ms_stage"],
                            "counters": {k: dna["stats"][k] for k in ("node_tests", "leaf_pairs", "candidates",
                                                                      "verified", "results")},
                            "plain_qps": dna.get("plain_qps"), "plain_queries": dna.get("plain_queries")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
