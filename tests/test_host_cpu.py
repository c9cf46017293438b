"""Host-side checks that need no GPU: input generators and bench.py's
command-line contract."""
import os
import subprocess
import sys

import numpy as np

from paper_2404_00966_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_gaussian_mixture_is_seeded_and_shaped():
    a = synth.gaussian_mixture(5, 500, 12, 4, -1.0, 1.0, 0.5, 7, 9)
    b = synth.gaussian_mixture(5, 500, 12, 4, -1.0, 1.0, 0.5, 7, 9)
    assert a["objects"].shape == (500, 12) and a["objects"].dtype == np.float32
    assert a["range_queries"].shape == (7, 12) and a["knn_queries"].shape == (9, 12)
    for k in ("objects", "range_queries", "knn_queries", "labels"):
        assert np.array_equal(a[k], b[k])
    c = synth.gaussian_mixture(6, 500, 12, 4, -1.0, 1.0, 0.5, 7, 9)
    assert not np.array_equal(a["objects"], c["objects"])
    # the object stream does not depend on how many queries are drawn
    d = synth.gaussian_mixture(5, 500, 12, 4, -1.0, 1.0, 0.5, 3, 0)
    assert np.array_equal(a["objects"], d["objects"])


def test_query_cap_keeps_leading_queries():
    full = synth.make_workload("l2_10k_d16")
    cut = synth.make_workload("l2_10k_d16", queries=13)
    assert np.array_equal(full["range_queries"][:13], cut["range_queries"])
    assert np.array_equal(full["knn_queries"][:13], cut["knn_queries"])


def test_dna_families_lengths_and_alphabet():
    d = synth.dna_families(3, 10, 20, 64, 128, 0.05, 3)
    chars, off = d["objects"]
    assert len(off) == 201 and off[0] == 0 and off[-1] == len(chars)
    assert set(np.unique(chars).tolist()) <= set(b"ACGT")
    lens = np.diff(off)
    assert lens.min() >= 40 and lens.max() <= 160
    qc, qo = d["queries"]
    assert len(qo) == 31
    again = synth.dna_families(3, 10, 20, 64, 128, 0.05, 3)
    assert np.array_equal(again["objects"][0], chars) and np.array_equal(again["queries"][0], qc)


def test_mutation_rate_zero_copies_seeds():
    d = synth.dna_families(9, 4, 5, 10, 20, 0.0, 1)
    chars, off = d["objects"]
    strs = [chars[off[i]:off[i + 1]].tobytes() for i in range(len(off) - 1)]
    for f in range(4):
        assert len(set(strs[5 * f:5 * f + 5])) == 1


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_myers_recurrences_match_dynamic_programme(tmp_path):
    """The device's bit-parallel Levenshtein recurrences (full width, and the
    banded one-word form used for cutoffs up to 63) are host-callable: compile
    them for the host and compare with the dynamic programme on random and
    mutated string pairs (exact distance within the cutoff, above it
    otherwise)."""
    exe = tmp_path / "myers_host"
    subprocess.run(["hipcc", "-O2", "-std=c++17", "--offload-host-only", "-x", "hip",
                    os.path.join(ROOT, "tests", "myers_host.cpp"), "-o", str(exe)], check=True,
                   capture_output=True)
    for seed in (1, 2):
        r = subprocess.run([str(exe), str(seed), "60000"], capture_output=True, text=True)
        assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
