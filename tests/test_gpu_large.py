"""GPU parity at the full size of the large sparse workload (1M x 2M,
power-law column counts, about 9M nonzeros) and for every column-slab count
of the A x and A' y products.

The oracle runs here in its OpenMP build (bitwise equal to the plain
build, a CPU test checks that), so the first 1000 iterations at full size
take about a minute of host time.  Iterates, averages and anchors are
compared element by element: the norm bound and the per-coordinate bound
|z_gpu,i - z_cpu,i| <= 1e-10 (|z_cpu,i| + ||z_cpu||_inf) of
tests/parity.py; integer fields of the check records exactly, float fields
of the records to 1e-9; products row by row within the summation-order
bound.  The step size is fixed from the bound |A|_2 <= sqrt(|A|_1 |A|_inf)
so that no power iteration runs on the CPU.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2105_12715_amd import lpgen
from tests.parity import assert_points_match

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_12715_amd import _lib
    _lib.load(build_if_missing=False)
    return _lib


@pytest.fixture(scope="module")
def large():
    return lpgen.large_powerlaw()


def to_np(t):
    return t.detach().cpu().numpy()


def assert_within_sum_bound(got, ref, lp, v, transpose=False):
    """Row sums of A v (or A' v) summed in different orders agree within
    the bound of any summation order: |a - b| <= 2 k u sum_j |a_ij v_j|
    for a row of k entries, u = 2^-53."""
    A = lp.scipy_csr()
    if transpose:
        A = A.T.tocsr()
    k = np.diff(A.indptr).astype(float)
    mag = abs(A) @ np.abs(v)
    bound = 2.0 * k * 2.0 ** -53 * mag
    err = np.abs(np.asarray(got) - np.asarray(ref))
    assert np.all(err <= bound), float(np.max(err - bound))


def norm_bound_eta(lp):
    A = abs(lp.scipy_csr())
    n1 = float(A.sum(axis=0).max())
    ninf = float(A.sum(axis=1).max())
    return 0.9 / np.sqrt(n1 * ninf)


def test_large_matvec(lib, large):
    lp = large
    _say("large matvec", lp.name)
    s = lib.Solver(lp, eta=norm_bound_eta(lp))
    o = oracle.Oracle(lp, eta=1.0)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(lp.n)
    y = rng.standard_normal(lp.m)
    assert_within_sum_bound(to_np(s.matvec(x)), o.matvec(x), lp, x)
    assert_within_sum_bound(to_np(s.matvec(y, transpose=True)), o.matvec_t(y), lp, y, True)


@pytest.mark.timeout(900)
def test_large_iterates_and_checks(lib, large):
    """The first 1000 iterations of the restarted method at full size (33
    checks, restarts among them): the iterates, averages and anchors at
    k = 1, 30, 60, 300 and 1000, and every check record."""
    lp = large
    eta = norm_bound_eta(lp)
    _say("large iterates", lp.name, eta)
    o = oracle.Oracle(lp, eta=eta, mode=oracle.MODE_ADAPTIVE, parallel=True)
    s = lib.Solver(lp, eta=eta, restart_mode=oracle.MODE_ADAPTIVE)
    done = 0
    for k in (1, 30, 60, 300, 1000):
        o.solve(k - done, 0.0)
        s.solve(k - done, 0.0)
        done = k
        _say("  compared at", k)
        for which in (0, 1, 2):
            xo, yo = o.get(which)
            xg, yg = (to_np(t) for t in s.get_iterate(which))
            assert_points_match(np.concatenate([xg, yg]), np.concatenate([xo, yo]), 1e-10,
                                f"k={k} point {which}")
    lo, lg = o.log(), s.check_log()
    assert lo.shape == lg.shape == (33, 14)
    np.testing.assert_array_equal(lg[:, [0, 1, 2, 9, 10, 11]], lo[:, [0, 1, 2, 9, 10, 11]])
    for col in (3, 4, 5, 6, 7, 8, 12):
        np.testing.assert_allclose(lg[:, col], lo[:, col], rtol=1e-9, atol=1e-300)
    assert lo[:, 9].sum() >= 2


# equal column counts: the first 4 MiB of x holds its share of the columns
# of the entries, under 60% in every case, so A keeps its slabs
@pytest.mark.parametrize("m,n,per_col", [
    (3000, 1_000_000, 2),    # two slabs
    (5000, 1_100_000, 1),    # four slabs
    (20_000, 4_300_000, 1),  # eight slabs
    (1, 1_000_000, 1),       # one row, two slabs
    (600_000, 1_000_000, 1), # two slabs of A and two of A'
])
def test_slab_counts_matvec_and_steps(lib, m, n, per_col):
    lp = lpgen.column_count_lp(17, m, n, per_col=per_col, bounds="mix")
    _say("slabs", m, n, per_col)
    eta = norm_bound_eta(lp)
    s = lib.Solver(lp, eta=eta)
    o = oracle.Oracle(lp, eta=eta)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    assert_within_sum_bound(to_np(s.matvec(x)), o.matvec(x), lp, x)
    assert_within_sum_bound(to_np(s.matvec(y, transpose=True)), o.matvec_t(y), lp, y, True)
    o.solve(31, 0.0)
    s.solve(31, 0.0)
    for which in (0, 1):
        xo, yo = o.get(which)
        xg, yg = (to_np(t) for t in s.get_iterate(which))
        assert_points_match(np.concatenate([xg, yg]), np.concatenate([xo, yo]), 1e-10,
                            f"point {which}")


def test_large_transpose_in_callers_order(lib, large):
    """The library keeps the columns sorted by count; A' comes back in the
    caller's column order, entry for entry."""
    lp = large
    s = lib.Solver(lp, eta=norm_bound_eta(lp))
    trp, tci, tv, perm = (t.cpu().numpy() for t in s.transpose_csr())
    e_rp, e_ci, e_v, e_perm = oracle.transpose(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.vals)
    np.testing.assert_array_equal(trp, e_rp)
    np.testing.assert_array_equal(tci, e_ci)
    np.testing.assert_array_equal(tv, e_v)
    np.testing.assert_array_equal(perm, e_perm)


def test_reordered_columns_keeping_slabs(lib):
    """Mild count skew (20% of the columns hold two entries): the columns are
    reordered but the first 4 MiB of x holds under 60% of the entries, so
    A x keeps its column slabs."""
    n = 1_100_000
    cnt = np.where(np.random.default_rng(21).random(n) < 0.2, 2, 1)
    lp = lpgen.column_count_lp(22, 5000, n, counts=cnt, bounds="mix")
    _say("reordered with slabs", lp.nnz)
    eta = norm_bound_eta(lp)
    s = lib.Solver(lp, eta=eta)
    o = oracle.Oracle(lp, eta=eta)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(n)
    y = rng.standard_normal(lp.m)
    assert_within_sum_bound(to_np(s.matvec(x)), o.matvec(x), lp, x)
    assert_within_sum_bound(to_np(s.matvec(y, transpose=True)), o.matvec_t(y), lp, y, True)
    o.solve(61, 0.0)
    s.solve(61, 0.0)
    for which in (0, 1, 2):
        xo, yo = o.get(which)
        xg, yg = (to_np(t) for t in s.get_iterate(which))
        assert_points_match(np.concatenate([xg, yg]), np.concatenate([xo, yo]), 1e-10,
                            f"point {which}")
    # a point set through the API comes back unchanged
    s.set_iterate(x, y)
    xg, yg = (to_np(t) for t in s.get_iterate(0))
    np.testing.assert_array_equal(xg, x)
    np.testing.assert_array_equal(yg, y)
