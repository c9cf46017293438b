"""Seeded synthetic inputs shaped like the GTS evaluation workloads.

This module draws random objects and queries and nothing else: it computes no
distance, no pivot, no bound and no search result.  Both the CPU oracle tests
and the GPU path take their inputs from here, so the two sides see the same
bytes.

Two object families stand in for the paper's datasets (Sec. 6.1, Table 2):

* Gaussian mixtures of float32 vectors (L2 metric) -- the role of the paper's
  low-dimensional T-Loc set and of vector data in general.
* Families of DNA strings over {A,C,G,T} (edit-distance metric) -- the role of
  the paper's DNA set (1M strings of length about 100).

Every draw uses numpy's PCG64 bit generator, with independent streams spawned
from one ``SeedSequence`` per workload (means, objects, range queries, kNN
queries), so adding a stream never perturbs another.
"""
from __future__ import annotations

import numpy as np

DNA_ALPHABET = np.frombuffer(b"ACGT", dtype=np.uint8)

_CHUNK_ROWS = 1 << 18  # rows drawn per normal() call; fixed so draws are reproducible


def _streams(seed: int, count: int):
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(seed).spawn(count)]


def _mixture_rows(gen, means, n, sigma):
    """n rows x = mu_c + sigma * N(0, I), component c uniform, cast to float32."""
    K, D = means.shape
    labels = gen.integers(0, K, size=n)
    out = np.empty((n, D), dtype=np.float32)
    for a in range(0, n, _CHUNK_ROWS):
        b = min(n, a + _CHUNK_ROWS)
        noise = gen.standard_normal((b - a, D))
        out[a:b] = (means[labels[a:b]] + sigma * noise).astype(np.float32)
    return out, labels


def gaussian_mixture(seed: int, n: int, dim: int, components: int, lo: float,
                     hi: float, sigma: float, n_range: int = 0, n_knn: int = 0):
    """Objects and queries from one Gaussian mixture.

    Means are uniform on [lo, hi]^dim (float64), every component has equal
    weight, and each row is the component mean plus isotropic noise of
    standard deviation ``sigma``, rounded to float32.  Range and kNN queries
    are fresh draws from the same mixture on streams of their own.

    Returns a dict with ``objects`` [n, dim] float32, ``range_queries``
    [n_range, dim], ``knn_queries`` [n_knn, dim] and the integer ``labels``.
    """
    g_means, g_obj, g_rq, g_kq = _streams(seed, 4)
    means = g_means.uniform(lo, hi, size=(components, dim))
    objects, labels = _mixture_rows(g_obj, means, n, sigma)
    rq, _ = _mixture_rows(g_rq, means, n_range, sigma)
    kq, _ = _mixture_rows(g_kq, means, n_knn, sigma)
    return {"objects": objects, "labels": labels, "range_queries": rq,
            "knn_queries": kq}


def _mutate(gen, seed_codes: np.ndarray, copies: int, rate: float):
    """``copies`` mutants of one seed string (codes 0..3).

    Each position independently, with probability ``rate``, receives one edit
    of a uniformly chosen kind: substitution by one of the three other bases,
    insertion of a uniform base before it, or deletion.  All random arrays are
    drawn for every position so the stream consumption does not depend on the
    outcome.  Returns a list of uint8 code arrays.
    """
    L = seed_codes.shape[0]
    hit = gen.random((copies, L)) < rate
    kind = gen.integers(0, 3, size=(copies, L))      # 0 sub, 1 ins, 2 del
    shift = gen.integers(1, 4, size=(copies, L))     # substitution offset
    ins = gen.integers(0, 4, size=(copies, L))       # inserted base
    base = np.broadcast_to(seed_codes, (copies, L))
    sub = hit & (kind == 0)
    insm = hit & (kind == 1)
    dele = hit & (kind == 2)
    first = np.where(sub, (base + shift) % 4, base)
    first = np.where(insm, ins, first)
    second = base
    pair = np.stack([first, second], axis=2).astype(np.uint8)
    keep = np.stack([~dele, insm], axis=2)
    lens = keep.sum(axis=(1, 2))
    flat = pair[keep]
    ends = np.cumsum(lens)
    return [flat[e - l:e] for e, l in zip(ends, lens)]


def dna_families(seed: int, n_seeds: int, per_seed: int, min_len: int,
                 max_len: int, rate: float, queries_per_seed: int = 0):
    """DNA strings in families: random seeds plus point-mutated copies.

    Seed lengths are uniform on {min_len..max_len}, bases i.i.d. uniform.
    Objects are ``per_seed`` mutants of every seed (seed-major order); queries
    are ``queries_per_seed`` further mutants of every seed drawn on a separate
    stream and then shuffled.  Strings are returned in the packed form the
    library takes: ``chars`` uint8 (ASCII A/C/G/T) and ``offsets`` int64
    [count + 1].
    """
    g_seed, g_obj, g_q, g_shuf = _streams(seed, 4)
    seeds = []
    for _ in range(n_seeds):
        L = int(g_seed.integers(min_len, max_len + 1))
        seeds.append(g_seed.integers(0, 4, size=L).astype(np.uint8))
    objs, qs = [], []
    for s in seeds:
        objs.extend(_mutate(g_obj, s, per_seed, rate))
    for s in seeds:
        if queries_per_seed:
            qs.extend(_mutate(g_q, s, queries_per_seed, rate))
    if qs:
        order = g_shuf.permutation(len(qs))
        qs = [qs[i] for i in order]
    return {"objects": pack_strings(objs), "queries": pack_strings(qs),
            "family": np.repeat(np.arange(n_seeds), per_seed)}


def pack_strings(codes_list):
    """List of code arrays (0..3) -> (chars as ASCII uint8, offsets int64)."""
    lens = np.array([len(c) for c in codes_list], dtype=np.int64)
    offsets = np.zeros(len(codes_list) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    if codes_list:
        codes = np.concatenate(codes_list) if offsets[-1] else np.zeros(0, np.uint8)
    else:
        codes = np.zeros(0, np.uint8)
    return DNA_ALPHABET[codes], offsets


def strings_from_bytes(items):
    """List of bytes objects -> packed (chars uint8, offsets int64)."""
    lens = np.array([len(s) for s in items], dtype=np.int64)
    offsets = np.zeros(len(items) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    chars = np.frombuffer(b"".join(items), dtype=np.uint8).copy()
    return chars, offsets


def random_strings(seed: int, count: int, min_len: int, max_len: int,
                   alphabet: bytes = b"ACGT"):
    """Independent uniform strings (lengths uniform on {min_len..max_len})."""
    (g,) = _streams(seed, 1)
    alpha = np.frombuffer(alphabet, dtype=np.uint8)
    items = []
    for _ in range(count):
        L = int(g.integers(min_len, max_len + 1))
        items.append(alpha[g.integers(0, len(alpha), size=L)].tobytes())
    return strings_from_bytes(items)


# ---------------------------------------------------------------------------
# The named workloads.  Sizes, seeds and parameters are the experiment
# configurations; the radii that depend on distance quantiles are not drawn
# here (they are statistics of distances, computed by the oracle).
# ---------------------------------------------------------------------------

WORKLOADS = {
    # 10k x 16 L2, 10 components on [-10,10], sigma 1; 5 pivots, fanout 8, leaf 64
    "l2_10k_d16": dict(kind="l2", seed=966001, n=10_000, dim=16, components=10,
                       lo=-10.0, hi=10.0, sigma=1.0, n_range=100, n_knn=100,
                       k=10, pivots=5, fanout=8, leaf=64,
                       range_quantile=1e-3),
    # 1M x 128 L2, 100 components on [-5,5], sigma 1; 16 pivots, fanout 16, leaf 256
    "l2_1m_d128": dict(kind="l2", seed=966002, n=1_000_000, dim=128,
                       components=100, lo=-5.0, hi=5.0, sigma=1.0,
                       n_range=10_000, n_knn=10_000, k=16, pivots=16,
                       fanout=16, leaf=256, range_quantile=1e-4),
    # 500k DNA strings, 1000 seeds x 500 mutants, lengths 64-128, 5% mutation;
    # 8 pivots, fanout 8, leaf size from the height rule; range r = 8
    "dna_500k": dict(kind="dna", seed=966003, n_seeds=1000, per_seed=500,
                     min_len=64, max_len=128, rate=0.05, queries_per_seed=10,
                     radius=8, pivots=8, fanout=8, leaf=0),
    # 4M x 96 L2, 1000 components, sigma 0.5; 16 pivots, fanout 2, leaf 512
    # (no tree shape is given for this batch: the leaf count, a power of the
    # fanout, sets the node filter's work; 8,192 leaves of about 490 objects
    # gave the shortest step of the shapes measured, fanout 16 with leaf 256
    # making 65,536 leaves of 61)
    "l2_4m_d96": dict(kind="l2", seed=966004, n=4_000_000, dim=96,
                      components=1000, lo=-5.0, hi=5.0, sigma=0.5,
                      n_range=0, n_knn=50_000, k=32, pivots=16, fanout=2,
                      leaf=512),
}


# Serving mix: an L2 index and a DNA index served together under an
# open-loop request trace.  Query pools and insert pools are fresh draws of the
# same distributions (held-out rows of the mixture, held-out mutants).
SERVING = {
    "serve_l2_2m_d128": dict(kind="l2", seed=966005, n=2_000_000, dim=128, components=100, lo=-5.0, hi=5.0,
                             sigma=1.0, query_pool=20_000, insert_pool=400_000, pivots=16, fanout=16, leaf=256),
    "serve_dna_200k": dict(kind="dna", seed=966006, n_seeds=400, per_seed=500, min_len=64, max_len=128,
                           rate=0.05, queries_per_seed=110, query_pool=4_000, pivots=8, fanout=8, leaf=0),
}


def make_serving(name: str):
    """Objects, a query pool and an insert pool of a serving index."""
    w = dict(SERVING[name])
    if w["kind"] == "l2":
        d = gaussian_mixture(w["seed"], w["n"] + w["insert_pool"], w["dim"], w["components"], w["lo"], w["hi"],
                             w["sigma"], w["query_pool"], 0)
        w.update(objects=d["objects"][:w["n"]], inserts=d["objects"][w["n"]:], queries=d["range_queries"])
        return w
    d = dna_families(w["seed"], w["n_seeds"], w["per_seed"], w["min_len"], w["max_len"], w["rate"],
                     w["queries_per_seed"])
    qc, qo = d["queries"]
    k = w["query_pool"]
    w.update(objects=d["objects"], queries=(qc[:qo[k]].copy(), qo[:k + 1].copy()),
             inserts=(qc[qo[k]:].copy(), (qo[k:] - qo[k]).copy()))
    return w


def make_workload(name: str, scale: float = 1.0, queries: int | None = None):
    """Draw a named workload.  ``scale`` < 1 shrinks the object count (and the
    family count for DNA) for quick tests; ``queries`` keeps only that many
    leading queries of each kind (the same rows the full draw starts with)."""
    w = dict(WORKLOADS[name])
    if w["kind"] == "l2":
        n = max(1, int(round(w["n"] * scale)))
        d = gaussian_mixture(w["seed"], n, w["dim"], w["components"], w["lo"],
                             w["hi"], w["sigma"], w["n_range"], w["n_knn"])
        if queries is not None:
            d["range_queries"] = d["range_queries"][:queries].copy()
            d["knn_queries"] = d["knn_queries"][:queries].copy()
        d.update(w)
        d["n"] = n
        return d
    ns = max(1, int(round(w["n_seeds"] * scale)))
    d = dna_families(w["seed"], ns, w["per_seed"], w["min_len"], w["max_len"],
                     w["rate"], w["queries_per_seed"])
    d.update(w)
    d["n_seeds"] = ns
    if queries is not None:
        chars, off = d["queries"]
        q = min(queries, len(off) - 1)
        d["queries"] = (chars[:off[q]].copy(), off[:q + 1].copy())
    return d
