"""The cost model of Sec. 5.3 (host arithmetic of libgts.so, no GPU): closed
forms worked by hand and the two regimes the paper discusses."""
import math
import os

import pytest

from paper_2404_00966_amd import gts


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gts.LIB_PATH):
        pytest.skip("libgts.so not built")
    return gts


def test_closed_forms(lib):
    # n = 4096, F = 16: three layers; sigma = 0 keeps every object (p = 1):
    #   1^2 * ceil(16/256) * 4^2 + 2^2 * ceil(256/256) * 4^2 + 3^2 * ceil(4096/256) * 4^2 = 16 + 64 + 2304
    assert lib.cost_model(4096, 16, 0.0, 1.0, 256.0) == pytest.approx(2384.0)
    # a bound that prunes everything (r^2 < 2 sigma^2: p = 0): one round per layer
    assert lib.cost_model(4096, 16, 10.0, 1.0, 256.0) == pytest.approx((1 + 4 + 9) * 16.0)
    # p = 1/2 (2 sigma^2 / r^2 = 1/2), F = 4, n = 64, C = 1: layers of 2, 4, 8
    assert lib.cost_model(64, 4, 0.25, 1.0, 1.0) == pytest.approx((1 * 2 + 4 * 4 + 9 * 8) * 4.0)
    # one object: one layer
    assert lib.cost_model(1, 8, 0.0, 1.0, 1000.0) == pytest.approx(9.0)
    for bad in ((0, 8, 0.0, 1.0, 10.0), (10, 1, 0.0, 1.0, 10.0), (10, 8, 0.0, 1.0, 0.0)):
        assert math.isnan(lib.cost_model(*bad))


def test_regimes(lib):
    # n << C: fewer layers win, a large fanout is preferred
    assert lib.cost_model(10_000, 64, 0.1, 1.0, 1e6) < lib.cost_model(10_000, 2, 0.1, 1.0, 1e6)
    # n >> C with weak pruning: a small fanout is preferred
    assert lib.cost_model(10**8, 2, 0.0, 1.0, 1e3) < lib.cost_model(10**8, 64, 0.0, 1.0, 1e3)
