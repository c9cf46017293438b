"""Benchmark: batched metric search on one MI355X.

Default workload (one step = one mixed batch through the whole search path):
  l2_1m_d128: 1,000,000 x 128 float32 vectors (100-component Gaussian
  mixture), 16 pivots, fanout 16, leaf 256; 10,000 kNN queries (k = 16) plus
  10,000 range queries at the 0.01% distance quantile, in one call.
Reported alongside in the same JSON line:
  dna_500k: 500,000 DNA strings (1,000 families x 500 mutants), 8 pivots,
    fanout 8; 10,000 range queries r = 8 per step;
  l2_4m_d96: 4,000,000 x 96 (1,000 components, sigma 0.5), 16 pivots,
    fanout 2, leaf 512; 50,000 kNN queries k = 32, bf16-guarded against
    float32 selection.

`value` is the device-resident rate: queries and index in HBM when the timed
region starts, answers left in device memory.  Each workload also reports
the rate with the queries handed over in pinned host memory and the answers
returned to host memory (PCIe included), the plain one-query-per-workgroup
form and the float32 selection over the same whole batch, and distance
evaluations per second.  Prints ONE JSON line.

`python bench.py --pmc-summary DIR_FETCH DIR_WRITE` turns two rocprofv3
counter runs (FETCH_SIZE, WRITE_SIZE) of this script into the HBM traffic
summary kept under profiles/ (read back here as `traffic`).
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
CSRC = os.path.join(ROOT, "paper_2404_00966_amd", "csrc")

METRIC = "queries/s oracle-exact: 1M×128 L2 kNN k=16, 500k DNA edit range r=8; p99 ms"
# MI355X published peaks
BF16_PEAK_TFLOPS = 2500.0       # dense bf16 MFMA
FP32_PEAK_TFLOPS = 157.3        # fp32 vector (FMA = 2 flop)
HBM_PEAK_GBS = 8000.0
# vector ALU: 256 CUs x 128 lanes per clock x 2.4 GHz = 78.6 T lane-ops/s,
# the rate the published fp32 vector peak counts (157.3 TFLOP/s, FMA = 2 flop).
# (One wave64 instruction per CU per clock, 39.3 T, is no ceiling: the edit
# verification's counters show 1.12 VALU instructions per busy CU-cycle.)
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12

# source files whose text decides each kernel's code (a profile's traffic
# figure is used only while they are unchanged)
KERNEL_SOURCES = {
    "k_verify_l2": ["k_final.hip"],
    "k_mfma_sweep": ["k_search.hip"],
    "k_bound_near": ["k_leaf.hip"],
    "k_bound_mfma": ["k_leaf.hip"],
    "k_leaf_box": ["k_search.hip"],
    "k_leaf_ball": ["k_leaf.hip"],
    "k_leaf_near": ["k_leaf.hip"],
    "k_l2_objfilter": ["k_filter32.hip"],
    "k_edit_objfilter": ["k_search.hip"],
    "k_verify_edit": ["k_final.hip"],
}
COMMON_SOURCES = ["dev_common.h", "kernels.h", "gts_internal.h"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_sha16(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel] + COMMON_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_traffic():
    """{workload: {kernel: entry}} from the JSON blocks of profiles/hbm_traffic__*.md."""
    out = {}
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic__*.md"))):
        text = open(path).read()
        for block in re.findall(r"```json\n(.*?)\n```", text, flags=re.S):
            try:
                d = json.loads(block)
            except ValueError:
                continue
            out.setdefault(d.get("workload", ""), {}).update(d.get("kernels", {}))
    return out


_TRAFFIC = None


def traffic(workload, kernel):
    """Measured HBM bytes per launch of `kernel` on `workload`, or None when no
    profile holds it or its source changed since the profile was taken."""
    global _TRAFFIC
    if _TRAFFIC is None:
        _TRAFFIC = profile_traffic()
    e = _profile_entry(workload, kernel)
    if not e or e.get("source_sha16") != source_sha16(kernel):
        return None
    return e.get("bytes")


def _profile_entry(workload, kernel):
    """A profile's entry for `kernel`, from a summary whose workload label
    (workloads joined by '+') names `workload`."""
    global _TRAFFIC
    if _TRAFFIC is None:
        _TRAFFIC = profile_traffic()
    for wl, ks in _TRAFFIC.items():
        if workload in wl.split("+") and kernel in ks:
            return ks[kernel]
    return None


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


def same_answers(a, b):
    """Element-by-element equality of two results (ids and distances)."""
    import torch

    return (torch.equal(a.offsets.cpu(), b.offsets.cpu()) and torch.equal(a.ids.cpu(), b.ids.cpu())
            and torch.equal(a.dist.cpu(), b.dist.cpu()))


def dist_evals(st, m):
    """Exact metric evaluations of one call: query-to-pivot distances, the
    kNN bound windows and the verified candidates (cache scans included)."""
    return st["nq"] * m + st["bound_evals"] + st["verified"]


def run_l2(args, gts, synth, torch, np):
    w = synth.WORKLOADS["l2_1m_d128"]
    radii = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))
    r = radii["l2_1m_d128"]["radius_f32"]
    t = time.perf_counter()
    d = synth.make_workload("l2_1m_d128", queries=args.queries)
    log(f"l2_1m_d128 generated in {time.perf_counter() - t:.1f}s")
    X = torch.from_numpy(d["objects"]).cuda()
    Qh = torch.from_numpy(np.concatenate([d["knn_queries"], d["range_queries"]])).pin_memory()
    Q = Qh.cuda()
    nk, nr = len(d["knn_queries"]), len(d["range_queries"])
    nq = nk + nr
    k = np.array([w["k"]] * nk + [0] * nr, np.int32)
    radius = np.full(nq, r, np.float32)
    torch.cuda.synchronize()
    t = time.perf_counter()
    idx = gts.Index(X, gts.L2_F32, num_pivots=w["pivots"], fanout=w["fanout"], leaf_size=w["leaf"],
                    seed=w["seed"])
    build_s = time.perf_counter() - t
    log(f"index built in {build_s:.1f}s: {idx.info()}")
    # let the index's query context settle its tuned knob (untimed)
    tune_calls = 0
    for tune_calls in range(1, 33):
        idx.search(Q, radius=radius, k=k, result="device")
        if idx.stats()["tuning"] == 0:
            break
    log(f"tuning finished after {tune_calls} calls")
    # one call with the bf16 bound self-check (untimed): every rechecked
    # candidate's float32 distance against its proven interval
    idx.search(Q, radius=radius, k=k, result="device", flags=gts.QF_CHECK_BOUND)
    check = idx.stats()
    total, per = timed_steps(lambda: idx.search(Q, radius=radius, k=k, result="device"), args.steps, args.warmup)
    ms = total * 1e3 / args.steps
    # one more step with stage timing on, for the stage split and the roofline
    idx.set_timing(True)
    ref = idx.search(Q, radius=radius, k=k, result="device")
    st = idx.stats()
    idx.set_timing(False)
    st["bound_violations"] = check["bound_violations"]
    st["bound_checked"] = check["verified"]
    out = {"qps": nq * args.steps / total, "ms_per_step": ms, "per_step_ms": per, "build_s": build_s,
           "stats": st, "nq": nq, "r": r, "k": w["k"], "n": d["n"], "dim": w["dim"], "m": w["pivots"],
           "tuned": {"bound_window": st["bound_window"], "sweep_grid_per_cu": st["sweep_grid_per_cu"],
                     "tuning_calls": tune_calls},
           "dist_evals_per_s": dist_evals(st, w["pivots"]) / (ms * 1e-3)}
    # the same batch as one recorded HIP graph (gts_plan_*): every stage on
    # the device, no host synchronisation inside a step
    if not args.no_graph:
        total_ans = int(ref.offsets[-1])
        plan = gts.Plan(idx, nq, capacity=total_ans + total_ans // 4 + 1024)
        plan.queries.copy_(Q)
        plan.radius.copy_(torch.from_numpy(radius).cuda())
        plan.k.copy_(torch.from_numpy(k).cuda())
        tg, perg = timed_steps(plan.launch, args.steps, args.warmup)
        got, gst = plan.result()
        out["graph_plan"] = {"qps": nq * args.steps / tg, "ms_per_step": tg * 1e3 / args.steps,
                             "p50_ms": pct(perg, 50), "p99_ms": pct(perg, 99), "status": gst,
                             "same_answers": same_answers(ref, got)}
        log(f"l2 graph plan: {out['graph_plan']}")
        plan.close()
    if args.side_steps > 0:
        # PCIe included: queries from pinned host memory, answers to host memory
        th, perh = timed_steps(lambda: idx.search(Qh, radius=radius, k=k, result="host"), args.side_steps, 1)
        out["host_to_host"] = {"qps": nq * args.side_steps / th, "ms_per_step": th * 1e3 / args.side_steps,
                               "p99_ms": pct(perh, 99)}
        # the same whole batch in the plain form and with float32 selection
        for name, kw in (("plain", {"mode": gts.MODE_PLAIN}), ("fp32_selection", {"precision": gts.FP32}),
                         ("no_prune", {"flags": gts.QF_NO_PRUNE})):
            res = []
            tp, _ = timed_steps(lambda: res.append(idx.search(Q, radius=radius, k=k, result="device", **kw)),
                                args.side_steps, 1)
            out[name] = {"qps": nq * args.side_steps / tp, "ms_per_step": tp * 1e3 / args.side_steps,
                         "same_answers": same_answers(ref, res[-1]),
                         "candidates": idx.stats()["candidates"], "verified": idx.stats()["verified"]}
            log(f"l2 {name}: {out[name]}")
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
    qch, qoh = torch.from_numpy(qc).pin_memory(), torch.from_numpy(qo).pin_memory()
    qct, qot = qch.cuda(), qoh.cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    idx = gts.Index((oc, oo), gts.EDIT_U8, num_pivots=w["pivots"], fanout=w["fanout"], seed=w["seed"])
    build_s = time.perf_counter() - t
    log(f"dna index built in {build_s:.1f}s: {idx.info()}")
    radius = np.full(nq, float(w["radius"]), np.float32)
    total, per = timed_steps(lambda: idx.search((qct, qot), radius=radius, result="device"), args.steps,
                             args.warmup)
    ms = total * 1e3 / args.steps
    idx.set_timing(True)
    ref = idx.search((qct, qot), radius=radius, result="device")
    st = idx.stats()
    idx.set_timing(False)
    out = {"qps": nq * args.steps / total, "ms_per_step": ms, "per_step_ms": per, "build_s": build_s,
           "stats": st, "nq": nq, "dist_evals_per_s": dist_evals(st, w["pivots"]) / (ms * 1e-3)}
    if args.side_steps > 0:
        th, perh = timed_steps(lambda: idx.search((qch, qoh), radius=radius, result="host"), args.side_steps, 1)
        out["host_to_host"] = {"qps": nq * args.side_steps / th, "ms_per_step": th * 1e3 / args.side_steps,
                               "p99_ms": pct(perh, 99)}
        res = []
        tp, _ = timed_steps(lambda: res.append(idx.search((qct, qot), radius=radius, mode=gts.MODE_PLAIN,
                                                          result="device")), max(1, args.side_steps // 2), 1)
        out["plain"] = {"qps": nq * max(1, args.side_steps // 2) / tp,
                        "ms_per_step": tp * 1e3 / max(1, args.side_steps // 2),
                        "same_answers": same_answers(ref, res[-1])}
        log(f"dna plain: {out['plain']}")
    idx.close()
    return out, d


def run_l4m(args, gts, synth, torch, np):
    """4M x 96, 50,000 kNN (k = 32): bf16-guarded selection against float32
    selection and the plain form on the whole batch, and the largest
    relative distance error of a sample of answers against float64."""
    w = synth.WORKLOADS["l2_4m_d96"]
    t = time.perf_counter()
    d = synth.make_workload("l2_4m_d96", queries=args.queries)
    log(f"l2_4m_d96 generated in {time.perf_counter() - t:.1f}s")
    X = d["objects"]
    KQ = d["knn_queries"]
    nq = len(KQ)
    idx = gts.Index(torch.from_numpy(X).cuda(), gts.L2_F32, num_pivots=w["pivots"], fanout=w["fanout"],
                    leaf_size=w["leaf"], seed=w["seed"])
    Q = torch.from_numpy(KQ).cuda()
    for _ in range(32):
        idx.knn(Q, w["k"], result="device")
        if idx.stats()["tuning"] == 0:
            break
    steps = max(2, args.side_steps)
    total, per = timed_steps(lambda: idx.knn(Q, w["k"], result="device"), steps, 1)
    idx.set_timing(True)
    ref = idx.knn(Q, w["k"], result="device")
    st = idx.stats()
    idx.set_timing(False)
    idx.knn(Q, w["k"], result="device", flags=gts.QF_CHECK_BOUND)
    st["bound_violations"] = idx.stats()["bound_violations"]
    st["bound_checked"] = idx.stats()["verified"]
    out = {"qps": nq * steps / total, "ms_per_step": total * 1e3 / steps, "p99_ms": pct(per, 99), "nq": nq,
           "k": w["k"], "pivots": w["pivots"], "fanout": w["fanout"], "leaf": w["leaf"],
           "n_leaves": idx.info()["n_leaves"], "stats": st}
    for name, kw in (("fp32_selection", {"precision": gts.FP32}), ("plain", {"mode": gts.MODE_PLAIN})):
        res = []
        tp, _ = timed_steps(lambda: res.append(idx.knn(Q, w["k"], result="device", **kw)), 1, 1)
        out[name] = {"qps": nq / tp, "ms_per_step": tp * 1e3, "same_answers": same_answers(ref, res[-1])}
        log(f"l2_4m_d96 {name}: {out[name]}")
    idx.close()
    lists = ref.to_lists()
    rng = np.random.default_rng(4)
    worst = 0.0
    for i in rng.choice(nq, 64, replace=False):
        ids, dist = lists[i]
        exact = np.sqrt(((X[ids].astype(np.float64) - KQ[i].astype(np.float64)) ** 2).sum(axis=1))
        worst = max(worst, float(np.max(np.abs(dist.astype(np.float64) - exact) / np.maximum(exact, 1e-30))))
    out["max_rel_err_vs_f64"] = worst
    out["rel_err_sample"] = "every answer of 64 random queries"
    return out


def run_update_sweep(args, gts, synth, torch, np):
    """Update cost against the cache-list limit (the paper's Table 5 set-up
    on synthetic data): per limit, U updates, each deleting a random live
    object, inserting it back (fresh id) and running one random range query;
    the index rebuilds whenever the cache list exceeds its limit.  Then the
    batch update: 10% of the objects deleted and inserted back in one
    gts_update_batch call (direct reconstruction)."""
    radii = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))
    out = {}
    sets = {}
    d = synth.gaussian_mixture(966101, args.update_n, 128, 100, -5.0, 5.0, 1.0, 256, 0)
    sets["l2_d128"] = (gts.L2_F32, d["objects"], d["range_queries"], radii["l2_1m_d128"]["radius_f32"],
                       dict(num_pivots=16, fanout=16, leaf_size=256))
    dd = synth.dna_families(966102, max(1, args.update_n // 500), 500, 64, 128, 0.05, 1)
    sets["dna"] = (gts.EDIT_U8, dd["objects"], dd["queries"], 8.0, dict(num_pivots=8, fanout=8))
    rng = np.random.default_rng(966103)
    for name, (metric, objs, queries, r, kw) in sets.items():
        if metric == gts.L2_F32:
            n = len(objs)
            obj = lambda i: objs[i:i + 1]
            qsel = lambda j: torch.from_numpy(queries[j:j + 1]).cuda()
            nqs = len(queries)
            dev_objs = torch.from_numpy(objs).cuda()
        else:
            chars, off = objs
            n = len(off) - 1
            obj = lambda i: (chars[off[i]:off[i + 1]], np.array([0, off[i + 1] - off[i]], np.int64))
            qc, qo = queries
            qsel = lambda j: (torch.from_numpy(qc[qo[j]:qo[j + 1]]).cuda(),
                              torch.from_numpy(np.array([0, qo[j + 1] - qo[j]], np.int64)).cuda())
            nqs = len(qo) - 1
            dev_objs = (torch.from_numpy(chars).cuda(), torch.from_numpy(off).cuda())
        rows = []
        for limit in args.update_limits:
            idx = gts.Index(dev_objs, metric, cache_limit=limit, seed=7, **kw)
            row_of = list(range(n))          # id -> source row
            live = list(range(n))
            t = time.perf_counter()
            for u in range(args.update_count):
                j = int(rng.integers(0, len(live)))
                victim = live[j]
                idx.delete([victim])
                src = row_of[victim]
                nid = int(idx.insert(obj(src))[0])
                live[j] = nid
                if nid >= len(row_of):
                    row_of.extend([0] * (nid + 1 - len(row_of)))
                row_of[nid] = src
                idx.range(qsel(int(rng.integers(0, nqs))), r, result="device")
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            rows.append({"cache_limit": limit, "updates": args.update_count,
                         "ms_per_update": el * 1e3 / args.update_count, "rebuilds": idx.info()["rebuilds"]})
            log(f"update sweep {name}: {rows[-1]}")
            idx.close()
        # batch update: 10% deleted and inserted back in one call
        idx = gts.Index(dev_objs, metric, seed=7, **kw)
        gone = rng.choice(n, n // 10, replace=False)
        if metric == gts.L2_F32:
            back = objs[gone]
        else:
            back = synth.strings_from_bytes([chars[off[i]:off[i + 1]].tobytes() for i in gone])
        torch.cuda.synchronize()
        t = time.perf_counter()
        idx.update_batch(back, gone)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t
        t = time.perf_counter()
        idx2 = gts.Index(dev_objs, metric, seed=7, **kw)
        torch.cuda.synchronize()
        tbuild = time.perf_counter() - t
        idx.close()
        idx2.close()
        out[name] = {"n": n, "sweep": rows, "batch_update_10pct_s": tb, "build_s": tbuild}
    return out


def run_fanout_sweep(args, gts, synth, torch, np):
    """The cost model's preferred fanout against measured throughput (the
    paper's node-capacity experiment on the 1M x 128 workload): per fanout,
    build, settle the tuner, time the mixed batch; beside it the model cost
    of a range query (sigma^2 from a seeded sample, r the workload radius)."""
    w = synth.WORKLOADS["l2_1m_d128"]
    r = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))["l2_1m_d128"]["radius_f32"]
    d = synth.make_workload("l2_1m_d128", queries=args.queries)
    X = torch.from_numpy(d["objects"]).cuda()
    Q = torch.from_numpy(np.concatenate([d["knn_queries"], d["range_queries"]])).cuda()
    nk, nr = len(d["knn_queries"]), len(d["range_queries"])
    k = np.array([w["k"]] * nk + [0] * nr, np.int32)
    radius = np.full(nk + nr, r, np.float32)
    best, costs = gts.choose_fanout(d["objects"], gts.L2_F32, r)
    rows = []
    for F in args.fanouts:
        t = time.perf_counter()
        idx = gts.Index(X, gts.L2_F32, num_pivots=w["pivots"], fanout=F, leaf_size=w["leaf"], seed=w["seed"])
        build_s = time.perf_counter() - t
        for _ in range(32):
            idx.search(Q, radius=radius, k=k, result="device")
            if idx.stats()["tuning"] == 0:
                break
        total, per = timed_steps(lambda: idx.search(Q, radius=radius, k=k, result="device"), args.steps, 1)
        rows.append({"fanout": F, "levels": idx.info()["levels"], "build_s": build_s,
                     "qps": (nk + nr) * args.steps / total, "model_cost": float(costs[F - 2])})
        log(f"fanout sweep: {rows[-1]}")
        idx.close()
    return {"model_choice": best, "rows": rows, "radius": r}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, l2data, dnadata, np):
    """The oracle (test infrastructure) on bounded samples of the same
    workloads, on the host cores: the float64 brute force on every core and
    on one core, the brute-force Wagner-Fischer on the DNA set, and the
    GTS-literal CPU tree search with its distance-evaluation counts."""
    import oracle as O

    radii = json.load(open(os.path.join(ROOT, "oracle", "radii.json")))
    r = radii["l2_1m_d128"]["radius_f32"]
    X = l2data["objects"]
    n = len(X)
    objs = O.ObjectSet(vecs=X)
    cores = O.set_threads(0)

    def l2_bf(m):
        kq = O.ObjectSet(vecs=np.ascontiguousarray(l2data["knn_queries"][:m]))
        rq = O.ObjectSet(vecs=np.ascontiguousarray(l2data["range_queries"][:m]))
        t = time.perf_counter()
        O.knn_bf(objs, kq, 16)
        O.range_bf(objs, rq, r)
        return time.perf_counter() - t

    m = args.cpu_queries // 2
    el = l2_bf(m)
    out = {"value": 2 * m / el, "unit": "queries/s", "cores": cores, "kind": "oracle",
           "sample": f"{m} kNN (k=16) + {m} range queries of l2_1m_d128 over all {n:,} x 128 objects, "
                     f"float64 brute force, {el:.1f}s",
           "cpu_model": cpu_model(), "dist_evals_per_s": 2 * m * n / el}
    m1 = max(1, args.cpu_queries // 100)
    O.set_threads(1)
    el1 = l2_bf(m1)
    O.set_threads(cores)
    out["one_core"] = {"value": 2 * m1 / el1, "cores": 1, "dist_evals_per_s": 2 * m1 * n / el1,
                       "sample": f"{m1} kNN + {m1} range queries, {el1:.1f}s"}
    # GTS-literal tree (Algorithms 1-5 on the CPU): build, then sampled queries
    t = time.perf_counter()
    tree = O.GtsTree(objs, 16, seed=1)
    tb = time.perf_counter() - t
    kq = O.ObjectSet(vecs=np.ascontiguousarray(l2data["knn_queries"][:m1]))
    rq = O.ObjectSet(vecs=np.ascontiguousarray(l2data["range_queries"][:m1]))
    t = time.perf_counter()
    _, ek = tree.knn(kq, 16)
    _, er = tree.range(rq, r)
    tt = time.perf_counter() - t
    ev = np.concatenate([ek, er])
    out["gts_tree"] = {"value": 2 * m1 / tt, "cores": 1, "build_s": tb,
                       "dist_evals_per_query": float(ev.mean()), "fraction_of_n": float(ev.mean() / n),
                       "dist_evals_per_s": float(ev.sum() / tt),
                       "sample": f"{m1} kNN + {m1} range queries, single-threaded, {tt:.1f}s"}
    if dnadata is not None:
        from paper_2404_00966_amd import synth

        chars, off = dnadata["objects"]
        qc, qo = dnadata["queries"]
        md = args.cpu_dna_queries if args.cpu_dna_queries > 0 else cores   # one round of the cores
        sc, so = synth.strings_from_bytes([qc[qo[i]:qo[i + 1]].tobytes() for i in range(md)])
        eo = O.ObjectSet(strings=(chars, off))
        t = time.perf_counter()
        O.range_bf(eo, O.ObjectSet(strings=(sc, so)), 8.0)
        ed = time.perf_counter() - t
        nd = len(off) - 1
        out["dna_500k"] = {"value": md / ed, "unit": "queries/s", "cores": cores,
                           "dist_evals_per_s": md * nd / ed,
                           "sample": f"{md} range queries (r=8) over all {nd:,} strings, full Wagner-Fischer, "
                                     f"{ed:.1f}s"}
    return out
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
    out["rebuild_ms"] = [il2.info()["rebuild_ms"], idna.info()["rebuild_ms"]]
    il2.close()
    idna.close()
    return out




def _roof(bound, achieved, peak, unit, work, launch_ms, what, traffic_bytes=None):
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak if achieved else None, "traffic": traffic_bytes, "work_per_launch": work,
            "launch_ms": launch_ms, "work": what}


def rooflines_l2(st, dim, workload):
    """Roofline points of the kernels behind the single-kernel stages of one
    search call (stage times are HIP-event times on the index's stream).
    Algorithmic work per launch:
      k_mfma_sweep: 2 * Dk flop (Dk = dim rounded up to 32) per (query,
        object) pair inside the surviving (query, leaf) pairs -- the method's
        own pairs; the dense-equivalent figure counts every pair of the
        computed (256-object slab, 16-query block) units instead;
      k_verify_l2: per candidate its 16-byte record and the 8 bytes of its
        norm and rounding error, per float32 recheck one object row (4 * dim
        bytes), per answer its 8-byte key;
      k_bound_mfma (with k_bound_near for the queries it leaves open): 2 * Dk
        flop per (query, window object) distance of the kNN bounds."""
    dk = (dim + 31) // 32 * 32
    ms = st["ms_stage"]
    out = {}
    t = ms["cands"]
    own = 2.0 * dk * st["own_pairs"]
    dense = 2.0 * dk * st["tile_pairs"] * 16 * 256
    a = own / (t * 1e-3) / 1e12 if t > 0 else None
    out["k_mfma_sweep"] = _roof("mfma", a, BF16_PEAK_TFLOPS, "TFLOP/s", own, t,
                                "2*Dk flop per (query, object) pair inside the surviving (query, leaf) pairs",
                                traffic(workload, "k_mfma_sweep"))
    ad = dense / (t * 1e-3) / 1e12 if t > 0 else None
    out["k_mfma_sweep"]["dense_equivalent"] = {
        "achieved": ad, "frac": ad / BF16_PEAK_TFLOPS if ad else None, "work_per_launch": dense,
        "work": "every pair of the computed (256-object slab, 16-query block) units, 2*Dk flop each"}
    t = ms["verify"]
    byts = 24.0 * st["candidates"] + 4.0 * dim * st["verified"] + 8.0 * st["results"]
    a = byts / (t * 1e-3) / 1e9 if t > 0 else None
    out["k_verify_l2"] = _roof("hbm", a, HBM_PEAK_GBS, "GB/s", byts, t,
                               "24 B per candidate + 4*dim B per float32 recheck + 8 B per answer",
                               traffic(workload, "k_verify_l2"))
    t = ms["bound"]
    fl = 2.0 * dk * st["bound_evals"]
    a = fl / (t * 1e-3) / 1e12 if t > 0 else None
    out["k_bound_mfma"] = _roof("mfma", a, BF16_PEAK_TFLOPS, "TFLOP/s", fl, t,
                                "2*Dk flop per (query, window object) distance of the kNN bounds (bf16 MFMA over "
                                "windows shared by 16-query blocks, and the exact windows of the queries those "
                                "leave open); the stage time covers both kernels",
                                traffic(workload, "k_bound_mfma"))
    return out


def rooflines_fp32_filter(st, mpad, workload):
    """k_l2_objfilter (float32 selection): per staged object its column of the
    pivot table (4 * mpad bytes) and 4 bytes of tombstone/position data, per
    candidate its 16-byte record; ALU work 3 * mpad per (query, object) test."""
    t = st["ms_stage"]["cands"]
    byts = (4.0 * mpad + 4.0) * st["filter_objects"] + 16.0 * st["candidates"]
    a = byts / (t * 1e-3) / 1e9 if t > 0 else None
    r = _roof("hbm", a, HBM_PEAK_GBS, "GB/s", byts, t,
              "(4*mpad + 4) B per staged object + 16 B per candidate", traffic("l2_1m_d128", "k_l2_objfilter"))
    ops = 3.0 * mpad * st["own_pairs"]
    ao = ops / (t * 1e-3) / 1e12 if t > 0 else None
    r["alu"] = {"achieved": ao, "peak": VALU_PEAK_TOPS, "unit": "Tops/s", "frac": ao / VALU_PEAK_TOPS if ao else None,
                "work_per_launch": ops, "work": "3*mpad VALU ops per (query, object) test"}
    return r


def rooflines_dna(st, mpad, workload):
    """k_edit_objfilter: per staged object its mpad-byte pivot-table row and 8
    bytes of offsets and tombstones, per candidate its 16-byte record;
    k_verify_edit is VALU-bound: its instruction count comes from the
    profiler (SQ_INSTS_VALU) when a fresh profile holds it."""
    out = {}
    t = st["ms_stage"]["cands"]
    byts = (mpad + 8.0) * st["filter_objects"] + 16.0 * st["candidates"]
    a = byts / (t * 1e-3) / 1e9 if t > 0 else None
    out["k_edit_objfilter"] = _roof("hbm", a, HBM_PEAK_GBS, "GB/s", byts, t,
                                    "(mpad + 8) B per staged object + 16 B per candidate",
                                    traffic(workload, "k_edit_objfilter"))
    t = st["ms_stage"]["verify"]
    e = _profile_entry(workload, "k_verify_edit") or {}
    insts = e.get("valu_insts") if e.get("source_sha16") == source_sha16("k_verify_edit") else None
    a = insts * 64 / (t * 1e-3) / 1e12 if insts and t > 0 else None
    out["k_verify_edit"] = _roof("alu", a, VALU_PEAK_TOPS, "T lane-ops/s", insts, t,
                                 "wave64 VALU instructions of the launch x 64 lanes (profile)",
                                 traffic(workload, "k_verify_edit"))
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


def _kernel_base(name):
    m = re.search(r"\b(k_[A-Za-z0-9_]+)", name)
    if m:
        return m.group(1)
    return "copy" if "copyBuffer" in name or "copy" in name.lower() else name[:40]


def _counter_rows(d):
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def pmc_summary(dirs, workload, last, command):
    """Markdown summary (with a JSON block bench.py reads back) of rocprofv3
    counter runs: per kernel the mean of its last `last` dispatches per
    counter, HBM bytes scaled by what FETCH_SIZE / WRITE_SIZE read for the
    256 MiB calibration copy."""
    per = {}     # (kernel, counter) -> [(dispatch, value)]
    for d in dirs:
        for r in _counter_rows(d):
            k = _kernel_base(r.get("Kernel_Name", ""))
            c = r.get("Counter_Name", "")
            per.setdefault((k, c), []).append((int(r.get("Dispatch_Id", 0)), float(r.get("Counter_Value", 0))))
    copy_bytes = 268435456.0
    factor = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        # the calibration copy is the first copy dispatch of the run
        # (--calibrate-copy runs before anything else touches the device)
        vals = sorted(per.get(("copy", c), []))
        if vals:
            factor[c] = copy_bytes / (vals[0][1] * 1024.0)
    kernels = {}
    for (k, c), vals in sorted(per.items()):
        if k == "copy" or k not in KERNEL_SOURCES:
            continue
        vals.sort()
        tail = [v for _, v in vals[-last:]]
        e = kernels.setdefault(k, {"source_sha16": source_sha16(k), "dispatches": len(vals)})
        key = {"FETCH_SIZE": "fetch_kib", "WRITE_SIZE": "write_kib", "SQ_INSTS_VALU": "valu_insts"}.get(c, c)
        e[key] = sum(tail) / len(tail)
    for k, e in kernels.items():
        if "fetch_kib" in e and "write_kib" in e and factor.get("FETCH_SIZE") and factor.get("WRITE_SIZE"):
            e["bytes"] = int(e["fetch_kib"] * 1024 * factor["FETCH_SIZE"] + e["write_kib"] * 1024 * factor["WRITE_SIZE"])
    lines = [f"# HBM traffic and counters per launch (rocprofv3 PMC): {workload}", "",
             "Commands (repository root, one MI355X), one counter group per run:", "", "```", *command, "```", "",
             "Calibration: one device copy of 268,435,456 bytes (`--calibrate-copy`); scale factors "
             + ", ".join(f"{c} x {v:.4f}" for c, v in factor.items()) + " (bytes per counted KiB / 1024).", "",
             f"Per launch: the mean of the last {last} dispatches of each kernel.  `bench.py` uses these figures as "
             "`traffic` only while the kernel's source hash matches `source_sha16`.", "",
             "| kernel | dispatches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | HBM bytes (MB) | SQ_INSTS_VALU |",
             "|---|---:|---:|---:|---:|---:|"]
    for k, e in sorted(kernels.items()):
        fk, wk, b, vi = e.get("fetch_kib"), e.get("write_kib"), e.get("bytes"), e.get("valu_insts")
        lines.append(f"| `{k}` | {e['dispatches']} | {fk if fk is None else f'{fk:,.1f}'} | "
                     f"{wk if wk is None else f'{wk:,.1f}'} | {b if b is None else f'{b / 1e6:,.1f}'} | "
                     f"{vi if vi is None else f'{vi:,.0f}'} |")
    other = sorted({c for e in kernels.values() for c in e
                    if c not in ("source_sha16", "dispatches", "fetch_kib", "write_kib", "valu_insts", "bytes")})
    if other:
        lines += ["", "Other counters per launch (same averaging):", "",
                  "| kernel | " + " | ".join(other) + " |", "|---|" + "---:|" * len(other)]
        for k, e in sorted(kernels.items()):
            if any(c in e for c in other):
                lines.append(f"| `{k}` | " + " | ".join("" if e.get(c) is None else f"{e[c]:,.0f}" for c in other)
                             + " |")
    lines += ["", "```json", json.dumps({"workload": workload, "copy_factor": factor, "kernels": kernels}, indent=1),
              "```", ""]
    return "\n".join(lines)


def _last_dispatches(d, last, top):
    """Per kernel, the mean duration of its last `last` dispatches in the
    run's kernel trace (kernel_trace.csv): with a run whose final calls are
    the timed steps, the figures of the launches the bench line reports."""
    per = {}
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
                per.setdefault(r["Kernel_Name"], []).append((t0, t1 - t0))
    rows = []
    for name, v in per.items():
        v.sort()
        tail = [x[1] for x in v[-last:]]
        rows.append((sum(tail) / len(tail), len(tail), min(tail), max(tail), name))
    rows.sort(key=lambda r: -r[0] * r[1])
    lines = ["", f"Last {last} dispatches of each kernel (the timed steps and the stage-timed call "
             "when they end the run):", "", "| kernel | dispatches | avg (us) | min (us) | max (us) |",
             "|---|---:|---:|---:|---:|"]
    for avg, n, lo, hi, name in rows[:top]:
        m = re.search(r"(k_[A-Za-z0-9_]+(<[^>]*>)?)", name)
        short = m.group(1) if m else name.split("(")[0][-60:]
        lines.append(f"| `{short}` | {n} | {avg / 1e3:,.1f} | {lo / 1e3:,.1f} | {hi / 1e3:,.1f} |")
    return lines


def stats_summary(d, title, command, top, last=0):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics: {title}", "", "Command (repository root, one MI355X):", "", "```",
             *command, "```", "", "| kernel | calls | avg (us) | min (us) | max (us) | total (ms) | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"]
        m = re.search(r"(k_[A-Za-z0-9_]+(<[^>]*>)?)", name)
        short = m.group(1) if m else name.split("(")[0][-60:]
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:,.1f} | {float(r['MinNs']) / 1e3:,.1f} | "
                     f"{float(r['MaxNs']) / 1e3:,.1f} | {float(r['TotalDurationNs']) / 1e6:,.2f} | "
                     f"{float(r['Percentage']):.1f} |")
    if last > 0:
        lines += _last_dispatches(d, last, top)
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--queries", type=int, default=None, help="cap queries per kind (default: full)")
    ap.add_argument("--side-steps", type=int, default=2,
                    help="steps of the host-to-host, plain and float32-selection legs (0: skip them)")
    ap.add_argument("--cpu-queries", type=int, default=800, help="L2 queries of the all-core oracle sample")
    ap.add_argument("--cpu-dna-queries", type=int, default=0, help="DNA oracle queries (0: one per core)")
    ap.add_argument("--skip-dna", action="store_true")
    ap.add_argument("--skip-c4", action="store_true", help="skip the 4M x 96 kNN leg")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay leg (profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true", help="run one 256 MiB device copy first (profiling)")
    ap.add_argument("--pmc-summary", nargs="+", metavar="DIR",
                    help="summarise rocprofv3 counter runs in DIR... (no GPU work)")
    ap.add_argument("--pmc-workload", default="l2_1m_d128")
    ap.add_argument("--pmc-last", type=int, default=2)
    ap.add_argument("--pmc-command", action="append", default=[])
    ap.add_argument("--stats-summary", metavar="DIR", help="summarise a rocprofv3 --stats run in DIR (no GPU work)")
    ap.add_argument("--stats-title", default="bench.py")
    ap.add_argument("--stats-top", type=int, default=40)
    ap.add_argument("--stats-last", type=int, default=0,
                    help="also list each kernel's mean over its last N dispatches (kernel trace)")
    ap.add_argument("--update-sweep", action="store_true",
                    help="update cost against the cache-list limit and the batch update, instead of the benchmark")
    ap.add_argument("--update-n", type=int, default=100000, help="objects of the update-sweep sets")
    ap.add_argument("--update-count", type=int, default=1000)
    ap.add_argument("--update-limits", type=int, nargs="+", default=[16, 64, 256, 1024, 4096])
    ap.add_argument("--fanout-sweep", action="store_true",
                    help="measured throughput against the cost model's fanout choice, instead of the benchmark")
    ap.add_argument("--fanouts", type=int, nargs="+", default=[4, 8, 16, 32, 64])
    ap.add_argument("--serving", action="store_true", help="run the serving mix instead of the batch benchmark")
    ap.add_argument("--serve-rate", type=float, default=50000.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-s", type=float, default=4.0, help="measured trace length, s")
    ap.add_argument("--serve-warmup-s", type=float, default=1.0)
    ap.add_argument("--serve-update-max", type=int, default=1000)
    ap.add_argument("--serve-lanes", type=int, default=2)
    ap.add_argument("--serve-cache", type=int, default=131072, help="cache list limit of the serving indexes")
    args = ap.parse_args()
    if args.pmc_summary:
        print(pmc_summary(args.pmc_summary, args.pmc_workload, args.pmc_last, args.pmc_command))
        return
    if args.stats_summary:
        print(stats_summary(args.stats_summary, args.stats_title, args.pmc_command, args.stats_top, args.stats_last))
        return
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
    if args.fanout_sweep:
        fs = run_fanout_sweep(args, gts, synth, torch, np)
        best = max(fs["rows"], key=lambda r: r["qps"])
        line = {"metric": "queries/s against the fanout (1M x 128 mixed batch)", "value": best["qps"],
                "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": None,
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16-mfma/f32",
                "data": "synthetic (seeded Gaussian mixture)",
                "config": {"workload": "fanout_sweep_l2_1m_d128", "fanouts": args.fanouts}, "fanout_sweep": fs}
        print(json.dumps(line), flush=True)
        return
    if args.update_sweep:
        us = run_update_sweep(args, gts, synth, torch, np)
        best = min(us["l2_d128"]["sweep"], key=lambda r: r["ms_per_update"])
        line = {"metric": "ms per streamed update (delete + reinsert + one range query), best cache-list limit",
                "value": best["ms_per_update"], "unit": "ms", "n_gpus": 1, "steps": args.update_count, "warmup": 0,
                "ms_per_step": best["ms_per_update"], "higher_is_better": False, "scaling": "weak",
                "vs_baseline": None, "dtype": "bf16-mfma/f32 (L2), int32 (edit)",
                "data": "synthetic (seeded mixture / DNA families)",
                "config": {"workload": "update_sweep", "n": args.update_n, "limits": args.update_limits},
                "update_sweep": us}
        print(json.dumps(line), flush=True)
        return
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
    dna, dnadata = None, None
    if not args.skip_dna:
        dna, dnadata = run_dna(args, gts, synth, torch, np)
        log(f"dna: {dna['qps']:.0f} q/s, {dna['ms_per_step']:.2f} ms/step, stages {dna['stats']['ms_stage']}")
    c4 = None
    if not args.skip_c4:
        c4 = run_l4m(args, gts, synth, torch, np)
        log(f"l2_4m_d96: {c4['qps']:.0f} q/s, {c4['ms_per_step']:.2f} ms/step")

    st = l2["stats"]
    roofs = rooflines_l2(st, l2["dim"], "l2_1m_d128")
    # the roofline reported is the one of the kernel that takes longest
    dom = max(roofs, key=lambda name: roofs[name]["launch_ms"])
    roof = dict(roofs[dom], kernel=dom)
    cpu = None
    if args.cpu_queries > 0:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args, l2data, dnadata, np)
    # the headline step is the recorded graph of the batch (gts_plan_*) when
    # its answers equal the eager call's; the eager call is reported beside it
    gp = l2.get("graph_plan")
    use_graph = bool(gp and gp["status"] == 0 and gp["same_answers"])
    eager = {"qps": l2["qps"], "ms_per_step": l2["ms_per_step"], "p50_ms": pct(l2["per_step_ms"], 50),
             "p99_ms": pct(l2["per_step_ms"], 99)}
    head = gp if use_graph else eager
    line = {
        "metric": METRIC,
        "value": head["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-mfma/f32",
        "data": "synthetic (seeded Gaussian mixture / DNA families)",
        "config": {"workload": "l2_1m_d128", "n": l2["n"], "dim": l2["dim"], "queries": l2["nq"],
                   "knn_k": l2["k"], "knn_queries": l2["nq"] // 2, "range_queries": l2["nq"] // 2,
                   "range_r": l2["r"], "pivots": 16, "fanout": 16, "leaf": 256},
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "latency_note": "batched: every query of a step completes with the step (makespan)",
        "value_note": ("one step = the whole batch through the recorded graph of a search plan (gts_plan_launch: "
                       "every stage on the device, no host synchronisation inside the step), answers identical to "
                       "the eager gts_search call (`eager`)" if use_graph else "one step = one eager gts_search call")
                      + "; queries and index resident in HBM, answers left in device memory; host_to_host hands "
                      "queries over in pinned host memory and returns answers to host memory",
        "dist_evals_per_s": l2["dist_evals_per_s"],
        "eager": eager,
        "host_to_host": l2.get("host_to_host"),
        "graph_plan": gp,
        "plain": l2.get("plain"),
        "fp32_selection": l2.get("fp32_selection"),
        "no_prune": l2.get("no_prune"),
        "stage_ms": st["ms_stage"],
        "counters": {k: st[k] for k in ("node_tests", "tile_pairs", "own_pairs", "candidates", "verified",
                                        "results", "bound_evals", "wide_queries", "bound_violations",
                                        "bound_checked")},
        "build_s": l2["build_s"],
        "tuned": l2["tuned"],
        "roofline": roof,
        "rooflines": roofs,
        "cpu_baseline": cpu,
    }
    if dna:
        dst = dna["stats"]
        line["dna_500k"] = {"queries_per_s": dna["qps"], "ms_per_step": dna["ms_per_step"],
                            "p50_ms": pct(dna["per_step_ms"], 50), "p99_ms": pct(dna["per_step_ms"], 99),
                            "queries": dna["nq"], "radius": 8, "build_s": dna["build_s"],
                            "dist_evals_per_s": dna["dist_evals_per_s"], "stage_ms": dst["ms_stage"],
                            "counters": {k: dst[k] for k in ("leaf_pairs", "own_pairs", "filter_objects",
                                                             "candidates", "verified", "results", "wide_queries")},
                            "host_to_host": dna.get("host_to_host"), "plain": dna.get("plain"),
                            "rooflines": rooflines_dna(dst, 8, "dna_500k")}
    if c4:
        line["l2_4m_d96"] = {k: v for k, v in c4.items() if k != "stats"}
        line["l2_4m_d96"]["stage_ms"] = c4["stats"]["ms_stage"]
        line["l2_4m_d96"]["counters"] = {k: c4["stats"][k] for k in ("own_pairs", "candidates", "verified",
                                                                     "bound_violations", "bound_checked")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
