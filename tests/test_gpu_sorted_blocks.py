"""Layouts and launch shapes of the products that must not change a bit of
the results.

A's merge-path blocks stored sorted by column (the layout the A x products
use by default when the columns fit the packed word) against the plain row
order: each product lands in LDS at its place in the row order, so the row
sums add the same terms in the same order.  The same holds for 128 against
256 threads per workgroup: a row is reduced by the same number of lanes in
the same order whatever the workgroup size.  Iterates, check records and
products must be bitwise equal, including blocks longer than the LDS stage
(one dense row of 6000 entries).
"""
import sys

import numpy as np
import pytest

from paper_2105_12715_amd import lpgen

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


def dense_row_lp(seed=31, m=400, n=6000, per_col=3):
    """Row 0 holds an entry in every column (a block longer than the LDS
    stage); every column has per_col more entries at distinct rows 1..m-1."""
    rng = np.random.default_rng(seed)
    cols = np.repeat(np.arange(n), per_col)
    rows = np.concatenate([rng.choice(np.arange(1, m), per_col, replace=False)
                           for _ in range(n)])
    rows = np.concatenate([np.zeros(n, np.int64), rows])
    cols = np.concatenate([np.arange(n), cols])
    vals = rng.standard_normal(rows.size)
    return lpgen.planted_lp(rng, m, n, rows, cols, vals, np.zeros(n), np.ones(n),
                            name="dense_row")


CASES = {
    "powerlaw": lambda: lpgen.column_count_lp(3, 3000, 7000, counts="powerlaw2",
                                              values="loguniform", bounds="mix"),
    "dense_row": dense_row_lp,
    "medium20kx50k": lambda: lpgen.medium(2),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_sorted_blocks_bitwise_equal(lib, name, monkeypatch):
    lp = CASES[name]()
    _say(f"[sorted-blocks] {name}: m={lp.m} n={lp.n} nnz={lp.nnz}")
    out = {}
    for mode in ("sorted", "plain"):
        if mode == "plain":
            monkeypatch.setenv("PDHG_SORTED_BLOCKS", "0")
        else:
            monkeypatch.delenv("PDHG_SORTED_BLOCKS", raising=False)
        monkeypatch.setenv("PDHG_TINY", "0")
        s = lib.Solver(lp, eta=0.0)
        r = s.solve(600, 0.0)
        x, y = (t.cpu().numpy() for t in s.get_iterate(lib.POINT_CURRENT))
        xa, ya = (t.cpu().numpy() for t in s.get_iterate(lib.POINT_AVERAGE))
        v = np.random.default_rng(5).standard_normal(lp.n)
        ax = s.matvec(torch.from_numpy(v).to("cuda")).cpu().numpy()
        out[mode] = (r, s.info()["eta"], x, y, xa, ya, ax, s.check_log())
        s.close()
    a, b = out["sorted"], out["plain"]
    assert a[0]["k"] == b[0]["k"] and a[0]["restarts"] == b[0]["restarts"]
    assert a[1] == b[1], "power iteration (A'A products) differs"
    for k, what in ((2, "x"), (3, "y"), (4, "x-bar"), (5, "y-bar"), (6, "A v")):
        assert np.array_equal(a[k], b[k]), f"{name}: {what} differs between layouts"
    assert np.array_equal(np.asarray(a[7]), np.asarray(b[7])), "check records differ"


@pytest.mark.parametrize("name", sorted(CASES))
def test_threads_per_workgroup_bitwise_equal(lib, name, monkeypatch):
    lp = CASES[name]()
    _say(f"[threads] {name}: m={lp.m} n={lp.n} nnz={lp.nnz}")
    out = {}
    monkeypatch.setenv("PDHG_TINY", "0")
    for wg in ("256", "128"):
        monkeypatch.setenv("PDHG_SPMV_WG", wg)
        s = lib.Solver(lp, eta=0.0)
        r = s.solve(600, 0.0)
        x, y = (t.cpu().numpy() for t in s.get_iterate(lib.POINT_CURRENT))
        v = np.random.default_rng(6).standard_normal(lp.m)
        aty = s.matvec(torch.from_numpy(v).to("cuda"), transpose=True).cpu().numpy()
        out[wg] = (r, x, y, aty, s.check_log())
        s.close()
    a, b = out["256"], out["128"]
    assert a[0]["k"] == b[0]["k"] and a[0]["restarts"] == b[0]["restarts"]
    for k, what in ((1, "x"), (2, "y"), (3, "A'v")):
        assert np.array_equal(a[k], b[k]), f"{name}: {what} differs between 256 and 128 threads"
    assert np.array_equal(np.asarray(a[4]), np.asarray(b[4])), "check records differ"


def empty_columns_lp(seed=41, m=20000, n=40000):
    """Column counts 0 (5%), 1 (40%), 2 (25%) and 3..20, >= rows and every
    bound class: with two slabs of y every column region is populated, and
    the empty columns (rows of A' with no entry in any slab) come last."""
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    counts = np.where(u < 0.05, 0, np.where(u < 0.45, 1, np.where(u < 0.70, 2,
                      rng.integers(3, 21, n))))
    return lpgen.column_count_lp(seed, m, n, counts=counts, bounds="mixed_inf",
                                 ge_frac=0.3, name="empty_cols")


@pytest.mark.parametrize("slab_bytes", ["65536", "131072"])
def test_slab_row_ranges_follow_the_oracle(lib, slab_bytes, monkeypatch):
    """Column slabs whose launches cover only the rows with entries in them
    (the update fused into each row's last launch) and launches over every
    row.  The merge-path blocks differ between the two, and with them the
    lanes that reduce a row, so the sums may round differently: both must
    give products within the summation-order bound and iterates that follow
    the oracle over 600 iterations with restarts.  Small slab slices force
    slabs: 65536 bytes gives the medium LP four slabs of y for A'y and eight
    of x for A x; 131072 bytes gives a 20,000 x 40,000 LP with empty
    columns, >= rows and every bound class two slabs of y (the columns then
    go in three regions by the slabs their rows fall in, then the empty
    ones) and four of x."""
    import oracle
    from tests.parity import assert_points_match, assert_within_sum_bound
    lp = lpgen.medium(2) if slab_bytes == "65536" else empty_columns_lp()
    A = abs(lp.scipy_csr())
    eta = 0.9 / np.sqrt(float(A.sum(axis=0).max()) * float(A.sum(axis=1).max()))
    o = oracle.Oracle(lp, eta=eta)
    o.solve(600, 0.0)
    v = np.random.default_rng(7).standard_normal(lp.m)
    u = np.random.default_rng(8).standard_normal(lp.n)
    monkeypatch.setenv("PDHG_TINY", "0")
    monkeypatch.setenv("PDHG_SLAB_BYTES", slab_bytes)
    for mode in ("ranges", "all"):
        if mode == "all":
            monkeypatch.setenv("PDHG_SLAB_RANGES", "0")
        else:
            monkeypatch.delenv("PDHG_SLAB_RANGES", raising=False)
        s = lib.Solver(lp, eta=eta)
        assert_within_sum_bound(s.matvec(torch.from_numpy(u).to("cuda")).cpu().numpy(),
                                o.matvec(u), A, u, f"{mode} A u")
        assert_within_sum_bound(s.matvec(torch.from_numpy(v).to("cuda"), transpose=True)
                                .cpu().numpy(), o.matvec_t(v), A.T.tocsr(), v, f"{mode} A'v")
        r = s.solve(600, 0.0)
        _say(f"[slab ranges] {slab_bytes} {mode}: k {r['k']} restarts {r['restarts']}")
        assert r["restarts"] == o.info()["restarts"]
        for which in (0, 1, 2):
            xo, yo = o.get(which)
            xg, yg = (t.cpu().numpy() for t in s.get_iterate(which))
            assert_points_match(np.concatenate([xg, yg]), np.concatenate([xo, yo]), 1e-10,
                                f"{slab_bytes} {mode} point {which}")
        s.close()
