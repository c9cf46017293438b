"""The no-allocation search (gts_search_noalloc) through the C ABI against
gts_search on the same index and queries: identical answers (ids and
distances, element by element) on two calls in a row, the second with a
smaller batch, for both metrics; and its error paths."""
import numpy as np
import pytest

from paper_2404_00966_amd import synth

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


def _same(res_a, res_b):
    a, b = res_a.to_lists(), res_b.to_lists()
    assert len(a) == len(b)
    for q, ((i1, d1), (i2, d2)) in enumerate(zip(a, b)):
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2), (q, i1[:5], i2[:5])


def test_noalloc_matches_search_l2(gts):
    d = synth.gaussian_mixture(301, 30000, 64, 25, -5.0, 5.0, 1.0, 900, 900)
    X = d["objects"]
    Q = np.concatenate([d["range_queries"], d["knn_queries"]])
    print("[case] no-alloc L2 1800 then 250 queries", flush=True)
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=8, fanout=8, leaf_size=64, seed=7)
    k = np.array([0] * 900 + [12] * 900, np.int32)
    radius = np.full(1800, 7.5, np.float32)
    for sel in (slice(0, 1800), slice(700, 950)):
        Qd = _dev(Q[sel])
        ref = idx.search(Qd, radius=radius[sel], k=k[sel], result="device")
        got, total = idx.search_noalloc(Qd, radius=radius[sel], k=k[sel], capacity=200 * (sel.stop - sel.start))
        assert total == int(ref.offsets[-1])
        _same(got, ref)
    idx.close()


def test_noalloc_matches_search_edit(gts):
    dd = synth.dna_families(302, 40, 120, 60, 100, 0.05, 10)
    chars, off = dd["objects"]
    qc, qo = dd["queries"]
    nq = len(qo) - 1
    print(f"[case] no-alloc edit {nq} then {nq // 3} queries", flush=True)
    idx = gts.Index((_dev(chars), _dev(off)), gts.EDIT_U8, num_pivots=6, fanout=6, seed=3)
    for m in (nq, nq // 3):
        Qd = (_dev(qc[:qo[m]]), _dev(qo[:m + 1]))
        k = np.array([0, 6] * (m // 2) + [0] * (m % 2), np.int32)
        radius = np.full(m, 6.0, np.float32)
        ref = idx.search(Qd, radius=radius, k=k, result="device")
        got, total = idx.search_noalloc(Qd, radius=radius, k=k, capacity=20000)
        assert total == int(ref.offsets[-1])
        _same(got, ref)
    idx.close()


def test_noalloc_errors(gts):
    d = synth.gaussian_mixture(303, 5000, 16, 5, -5.0, 5.0, 1.0, 64, 0)
    X, Q = d["objects"], d["range_queries"]
    print("[case] no-alloc errors", flush=True)
    idx = gts.Index(_dev(X), gts.L2_F32, num_pivots=4, fanout=4, leaf_size=32, seed=1)
    ref = idx.range(_dev(Q), 6.0, result="device")
    need = int(ref.offsets[-1])
    assert need > 1
    # answers beyond the output capacity: ENOMEM, with the count reported
    with pytest.raises(gts.GtsError) as e:
        idx.search_noalloc(_dev(Q), radius=6.0, capacity=need - 1)
    assert e.value.status == gts.ENOMEM
    # more queries than the entry point takes
    big = _dev(np.zeros((2049, 16), np.float32))
    with pytest.raises(gts.GtsError) as e:
        idx.search_noalloc(big, radius=1.0)
    assert e.value.status == gts.EINVAL
    # then a good call still matches
    got, total = idx.search_noalloc(_dev(Q), radius=6.0, capacity=need)
    assert total == need
    _same(got, ref)
    # an empty batch
    got, total = idx.search_noalloc(_dev(np.zeros((0, 16), np.float32)), radius=1.0)
    assert total == 0 and int(got.offsets[0]) == 0
    idx.close()
