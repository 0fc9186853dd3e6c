"""The OpenMP build of the oracle (same source, -DORC_OPENMP) gives bitwise
the results of the plain build: its parallel loops write only their own
outputs and its A'y sums each column in increasing row, the order the plain
build accumulates in; every reduction stays sequential.  This is what lets
the all-cores CPU baseline stand for the oracle."""
import numpy as np
import pytest

import oracle
from paper_2105_12715_amd import lpgen


@pytest.mark.parametrize("mode,method", [(oracle.MODE_ADAPTIVE, oracle.METHOD_PDHG),
                                         (oracle.MODE_FLEXIBLE, oracle.METHOD_PDHG),
                                         (oracle.MODE_FIXED, oracle.METHOD_PDHG),
                                         (oracle.MODE_ADAPTIVE, oracle.METHOD_EGM)])
def test_openmp_build_is_bitwise_equal(mode, method):
    lp = lpgen.column_count_lp(3, 3000, 7000, counts="powerlaw2", values="loguniform",
                               bounds="mix", ge_frac=0.3)
    a = oracle.Oracle(lp, mode=mode, method=method, fixed_len=50)
    b = oracle.Oracle(lp, mode=mode, method=method, fixed_len=50, parallel=True)
    assert a.info() == b.info()  # power iteration included
    ra = a.solve(900, 1e-7)
    rb = b.solve(900, 1e-7)
    for key in ("status", "k", "restarts", "which"):
        assert ra[key] == rb[key]
    for key in ("kkt", "pobj", "dobj"):
        assert ra[key] == rb[key] or (np.isnan(ra[key]) and np.isnan(rb[key]))
    np.testing.assert_array_equal(ra["x"], rb["x"])
    np.testing.assert_array_equal(ra["y"], rb["y"])
    for which in (0, 1, 2, 3):
        xa, ya = a.get(which)
        xb, yb = b.get(which)
        np.testing.assert_array_equal(xa, xb)
        np.testing.assert_array_equal(ya, yb)
    np.testing.assert_array_equal(a.log(), b.log())
    rng = np.random.default_rng(5)
    y = rng.standard_normal(lp.m)
    np.testing.assert_array_equal(a.matvec_t(y), b.matvec_t(y))


def test_openmp_build_uses_threads():
    assert oracle.threads(parallel=False) == 1
    assert oracle.threads(parallel=True) >= 1
