"""CPU: the multi-core oracle driver (used for the benchmark's CPU baseline)
renders the plain oracle's frame: per-trace bands added in trace order equal
the single sum to rounding, bit for bit across thread counts."""
import numpy as np
import pytest

import oracle
from workloads import Request, scene


@pytest.mark.parametrize("name", ["mini_table", "mini_sep", "c0"])
def test_omp_equals_plain(name):
    sc = scene(name)
    rq = Request(rv_mps=2.5, flux_scale=1.3)
    ref = oracle.render(sc, rq)
    a = oracle.render_omp(sc, rq, threads=1)
    b = oracle.render_omp(sc, rq, threads=3)
    c = oracle.render_omp(sc, rq, threads=8)
    # the fixed (trace) order makes the result independent of the thread count
    assert np.array_equal(a, b) and np.array_equal(a, c)
    # and equal to the plain scatter up to the rounding of partial sums
    assert np.max(np.abs(a - ref)) <= 1e-13 * np.max(ref)
    assert abs(a.sum() - ref.sum()) <= 1e-12 * ref.sum()
