"""pdhg_autotune: per-matrix choice of the column slabs, lanes per row and
threads per workgroup of A x and A'y.
The tuner times the products only, so the solver state stays bitwise the
same; solves after a re-slabbing still match the oracle; a second handle on
the same matrix takes the remembered choice.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2105_12715_amd import lpgen
from tests.parity import assert_points_match, assert_within_sum_bound

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


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def _eta(lp):
    A = abs(lp.scipy_csr())
    return 0.9 / np.sqrt(float(A.sum(axis=0).max()) * float(A.sum(axis=1).max()))


def test_autotune_keeps_state_and_parity(lib):
    # x of 8 MB and y of 4.8 MB: both products may use slabs
    lp = lpgen.column_count_lp(17, 600_000, 1_000_000, per_col=1, bounds="mix")
    eta = _eta(lp)
    _say("autotune", lp.nnz)
    s = lib.Solver(lp, eta=eta)
    o = oracle.Oracle(lp, eta=eta)
    s.solve(31, 0.0)
    o.solve(31, 0.0)
    before = [t.clone() for w in (0, 1, 2) for t in s.get_iterate(w)]
    info0 = s.info()
    r = s.autotune(iters=5, use_cache=False)
    _say(r)
    assert not r["from_cache"]
    assert sorted(r["A"]) == [1, 2, 4, 8] and sorted(r["At"]) == [1, 2, 4, 8]
    assert all(v > 0 for v in list(r["A"].values()) + list(r["At"].values()))
    assert r["slabs_A"] == min(r["A"], key=r["A"].get)
    assert r["slabs_At"] == min(r["At"], key=r["At"].get)
    assert sorted(r["lanes_A"]) == [-1, 0, 1] and sorted(r["lanes_At"]) == [-1, 0, 1]
    assert r["lanes_bias_A"] == min(r["lanes_A"], key=r["lanes_A"].get)
    assert r["lanes_bias_At"] == min(r["lanes_At"], key=r["lanes_At"].get)
    assert sorted(r["ms_threads_A"]) == [128, 256] and sorted(r["ms_threads_At"]) == [128, 256]
    assert r["threads_A"] == min(r["ms_threads_A"], key=r["ms_threads_A"].get)
    assert r["threads_At"] == min(r["ms_threads_At"], key=r["ms_threads_At"].get)
    after = [t for w in (0, 1, 2) for t in s.get_iterate(w)]
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(before, after))
    info1 = s.info()
    for key in ("k", "t", "restarts", "checks"):
        assert info0[key] == info1[key]
    # every slab count gives the same products up to rounding
    rng = np.random.default_rng(4)
    x = rng.standard_normal(lp.n)
    y = rng.standard_normal(lp.m)
    np.testing.assert_allclose(s.matvec(x).cpu().numpy(), o.matvec(x), rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(s.matvec(y, transpose=True).cpu().numpy(), o.matvec_t(y),
                               rtol=1e-12, atol=1e-9)
    # iterations after the re-slabbing still follow the oracle
    s.solve(61, 0.0)
    o.solve(61, 0.0)
    for which in (0, 1, 2):
        xo, yo = o.get(which)
        xg, yg = (t.cpu().numpy() for t in s.get_iterate(which))
        assert_points_match(np.concatenate([xg, yg]), np.concatenate([xo, yo]), 1e-10,
                            f"point {which}")
    # the same matrix again: the remembered choice, no timing
    s2 = lib.Solver(lp, eta=eta)
    r2 = s2.autotune(iters=5)
    assert r2["from_cache"] and r2["A"] == {} and r2["At"] == {}
    assert (r2["slabs_A"], r2["slabs_At"]) == (r["slabs_A"], r["slabs_At"])
    assert (r2["lanes_bias_A"], r2["lanes_bias_At"]) == (r["lanes_bias_A"], r["lanes_bias_At"])
    assert (r2["threads_A"], r2["threads_At"]) == (r["threads_A"], r["threads_At"])


@pytest.mark.parametrize("name", ["powerlaw", "medium"])
def test_every_lanes_bias_follows_the_oracle(lib, name):
    """Each lanes-per-row bias of both products (the row split the tuner
    chooses) gives products within the summation-order bound and iterates
    that follow the oracle over 300 iterations with restarts."""
    lp = (lpgen.column_count_lp(3, 3000, 7000, counts="powerlaw2", values="loguniform",
                                bounds="mix") if name == "powerlaw" else lpgen.medium(2))
    eta = _eta(lp)
    absA = abs(lp.scipy_csr())
    rng = np.random.default_rng(5)
    x = rng.standard_normal(lp.n)
    y = rng.standard_normal(lp.m)
    o = oracle.Oracle(lp, eta=eta)
    o.solve(300, 0.0)
    for bA in (-1, 0, 1):
        for bT in (-1, 0, 1):
            _say("lanes bias", name, bA, bT)
            s = lib.Solver(lp, eta=eta)
            s.set_schedule(1, 1, bA, bT)
            assert_within_sum_bound(s.matvec(x).cpu().numpy(), o.matvec(x), absA, x, "A x")
            assert_within_sum_bound(s.matvec(y, transpose=True).cpu().numpy(), o.matvec_t(y),
                                    absA.T.tocsr(), y, "A'y")
            s.solve(300, 0.0)
            for which in (0, 1, 2):
                xo, yo = o.get(which)
                xg, yg = (t.cpu().numpy() for t in s.get_iterate(which))
                assert_points_match(np.concatenate([xg, yg]), np.concatenate([xo, yo]), 1e-10,
                                    f"bias {bA},{bT} point {which}")
    s = lib.Solver(lp, eta=eta)
    for bad in [(3, 1, 0, 0), (1, 1, 2, 0), (1, 1, 0, -2)]:
        with pytest.raises(lib.PdhgError):
            s.set_schedule(*bad)


def test_autotune_without_slabs_and_bad_arguments(lib):
    lp = lpgen.small_dense(1)
    s = lib.Solver(lp, eta=0.1)
    r = s.autotune(iters=3, use_cache=False)
    assert (r["slabs_A"], r["slabs_At"]) == (1, 1) and r["A"] == {} and r["At"] == {}
    assert sorted(r["lanes_A"]) == [-1, 0, 1]
    with pytest.raises(lib.PdhgError):
        s.autotune(iters=0)
