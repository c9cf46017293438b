"""Write oracle/radii.json: range radii defined by distance quantiles.

A workload's range radius is the nearest-rank quantile of FP64 query-object
distances (the ceil(p * N)-th smallest of N pairs), rounded to float32 -- the
value both the oracle and the GPU library then use.  Only oracle/ computes
distances here.

  l2_10k_d16 : p = 0.1%  over all 100 range queries x all 10,000 objects
  l2_1m_d128 : p = 0.01% over the first 1,000 range queries x every 10th
               object (100,000), i.e. the 10,000th smallest of 1e8 pairs

Serving-mix tables (selectivity -> radius), from the query pool against a
strided sample of the objects:
  serve_l2_2m_d128 : radius at each selectivity of a log grid on
                     [1e-5, 1e-3], 500 queries x every 20th object (1e5)
  serve_dna_200k   : fraction of pairs within r for r = 0..40, 200 queries
                     x every 20th object (1e4); the serving radius for a
                     selectivity s is the largest r whose fraction is <= s
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from paper_2404_00966_amd import synth  # noqa: E402

RECIPES = {
    "l2_10k_d16": dict(queries=100, object_stride=1),
    "l2_1m_d128": dict(queries=1000, object_stride=10),
}


def radius_for(name):
    w = synth.WORKLOADS[name]
    rec = RECIPES[name]
    d = synth.make_workload(name)
    X = np.ascontiguousarray(d["objects"][::rec["object_stride"]])
    Q = np.ascontiguousarray(d["range_queries"][:rec["queries"]])
    D = O.pair_distances(O.ObjectSet(vecs=X), O.ObjectSet(vecs=Q)).ravel()
    rank = math.ceil(w["range_quantile"] * D.size)
    r64 = float(np.partition(D, rank - 1)[rank - 1])
    return {"quantile": w["range_quantile"], "pairs": int(D.size), "rank": rank,
            "queries": rec["queries"], "object_stride": rec["object_stride"],
            "radius_f64": r64, "radius_f32": float(np.float32(r64))}


def serving_tables():
    out = {}
    w = synth.make_serving("serve_l2_2m_d128")
    X = np.ascontiguousarray(w["objects"][::20])
    Q = np.ascontiguousarray(w["queries"][:500])
    D = O.pair_distances(O.ObjectSet(vecs=X), O.ObjectSet(vecs=Q)).ravel()
    D.sort()
    grid = np.logspace(-5, -3, 9)
    radii = [float(np.float32(D[max(math.ceil(s * D.size), 1) - 1])) for s in grid]
    out["serve_l2_2m_d128"] = {"pairs": int(D.size), "selectivity": grid.tolist(), "radius_f32": radii}
    w = synth.make_serving("serve_dna_200k")
    oc, oo = w["objects"]
    sub = list(range(0, len(oo) - 1, 20))
    items = [oc[oo[i]:oo[i + 1]].tobytes() for i in sub]
    X = O.ObjectSet(strings=synth.strings_from_bytes(items))
    qc, qo = w["queries"]
    Q = O.ObjectSet(strings=(qc[:qo[200]].copy(), qo[:201].copy()))
    D = O.pair_distances(X, Q).ravel()
    frac = [float(np.mean(D <= r)) for r in range(41)]
    out["serve_dna_200k"] = {"pairs": int(D.size), "within_r": frac}
    return out


def main():
    out = {name: radius_for(name) for name in RECIPES}
    out.update(serving_tables())
    path = os.path.join(HERE, "radii.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
