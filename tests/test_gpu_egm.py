"""GPU parity of restarted extragradient (eq. extra-gradient-update inside
Algorithm 1) against the oracle: iterates, target averages and anchors to a
relative 1e-10 over the first 1000 iterations, check records (integer
fields exactly, float fields to 1e-9), iteration counts of solves to 1e-8
exactly, and the column-slab products.
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


def rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


CASES = {
    "small50x100": lambda: lpgen.small_dense(1),
    "ge_rows": lambda: lpgen.bernoulli_lp(11, 30, 60, 0.15, lpgen.BOX01, ge_frac=0.4),
    "mixed_inf": lambda: lpgen.column_count_lp(13, 600, 1300, per_col=5,
                                               bounds="mixed_inf", ge_frac=0.5),
    "powerlaw": lambda: lpgen.column_count_lp(3, 3000, 7000, counts="powerlaw2",
                                              values="loguniform", bounds="mix"),
}


def _pair(lib, lp, mode, eta=None, **kw):
    if eta is None:
        eta = oracle.Oracle(lp).info()["eta"]
    o = oracle.Oracle(lp, eta=eta, mode=mode, method=oracle.METHOD_EGM, **kw)
    s = lib.Solver(lp, eta=eta, restart_mode=mode, method=lib.METHOD_EGM, **kw)
    return o, s


def _compare_points(o, s, tol=1e-10):
    for which in (0, 1, 2):
        xo, yo = o.get(which)
        xg, yg = (t.cpu().numpy() for t in s.get_iterate(which))
        assert_points_match(np.concatenate([xg, yg]), np.concatenate([xo, yo]), tol,
                            f"point {which}")


@pytest.mark.parametrize("name", list(CASES))
def test_egm_iterates_no_restart(lib, name):
    lp = CASES[name]()
    _say("egm none", name)
    o, s = _pair(lib, lp, oracle.MODE_NONE)
    done = 0
    for k in [1, 2, 7, 30, 31, 200, 1000]:
        o.step(k - done)
        s.step(k - done)
        done = k
        _compare_points(o, s)


@pytest.mark.parametrize("name,mode", [
    ("small50x100", oracle.MODE_ADAPTIVE), ("ge_rows", oracle.MODE_ADAPTIVE),
    ("mixed_inf", oracle.MODE_ADAPTIVE), ("powerlaw", oracle.MODE_ADAPTIVE),
    ("small50x100", oracle.MODE_FLEXIBLE), ("mixed_inf", oracle.MODE_FLEXIBLE),
])
def test_egm_iterates_and_checks_with_restarts(lib, name, mode):
    lp = CASES[name]()
    _say("egm restarts", name, mode)
    o, s = _pair(lib, lp, mode)
    done = 0
    for k in [30, 61, 300, 1000]:
        o.solve(k - done, 0.0)
        s.solve(k - done, 0.0)
        done = k
        _compare_points(o, s)
    lo, lg = o.log(), s.check_log()
    assert lo.shape == lg.shape == (33, 14)
    np.testing.assert_array_equal(lg[:, [0, 1, 2, 9, 10, 11]], lo[:, [0, 1, 2, 9, 10, 11]])
    for col in (3, 4, 5, 6, 7, 8, 12):
        np.testing.assert_allclose(lg[:, col], lo[:, col], rtol=1e-9, atol=1e-300)
    assert lo[:, 9].sum() >= 2


def test_egm_fixed_length_restarts(lib):
    lp = CASES["ge_rows"]()
    o, s = _pair(lib, lp, oracle.MODE_FIXED, fixed_len=64)
    for k in (63, 65, 640):
        o.solve(k, 0.0)
        s.solve(k, 0.0)
        _compare_points(o, s)


@pytest.mark.parametrize("name", ["small50x100", "ge_rows", "mixed_inf"])
def test_egm_solve_to_1e8_matches_oracle(lib, name):
    lp = CASES[name]()
    _say("egm solve", name)
    o, s = _pair(lib, lp, oracle.MODE_ADAPTIVE)
    ro = o.solve(400_000, 1e-8)
    rg = s.solve(400_000, 1e-8)
    assert ro["status"] == 0 and rg["status"] == 0
    assert rg["k"] == ro["k"] and rg["restarts"] == ro["restarts"]
    assert rg["which"] == ro["which"]
    np.testing.assert_allclose(rg["kkt"], ro["kkt"], rtol=1e-6)


def test_egm_over_column_slabs(lib):
    """A 600,000 x 1,000,000 LP splits both products into two slabs."""
    lp = lpgen.column_count_lp(17, 600_000, 1_000_000, per_col=1, bounds="mix")
    _say("egm slabs")
    A = abs(lp.scipy_csr())
    eta = 0.9 / np.sqrt(float(A.sum(axis=0).max()) * float(A.sum(axis=1).max()))
    o, s = _pair(lib, lp, oracle.MODE_ADAPTIVE, eta=eta)
    o.solve(31, 0.0)
    s.solve(31, 0.0)
    _compare_points(o, s)


def test_egm_kernel_timing_and_method_guards(lib):
    lp = CASES["powerlaw"]()
    o, s = _pair(lib, lp, oracle.MODE_ADAPTIVE)
    tp, td = s.time_iterations(20)
    assert tp > 0 and td > 0
    with pytest.raises(lib.PdhgError):
        lib.Solver(lp, method=7)


@pytest.mark.parametrize("name,iters", [("ge_rows", 300), ("mixed_inf", 120)])
def test_egm_weight_search(lib, name, iters):
    """The weight search with extragradient copies against independent
    oracle runs of the extragradient method."""
    lp = CASES[name]()
    eta = oracle.Oracle(lp).info()["eta"]
    om = [4.0 ** k for k in range(-5, 6)]
    s = lib.Solver(lp, eta=eta, method=lib.METHOD_EGM)
    kk, best, xg, yg = s.weight_search(om, iters, want_iterates=True)
    parts, obest, xo, yo = oracle.weight_search(lp, om, iters, eta, method=oracle.METHOD_EGM)
    xg, yg = xg.cpu().numpy(), yg.cpu().numpy()
    keys = ["kkt_rel", "primal_res", "dual_res", "pobj", "dobj", "kkt_paper_abs", "kkt_max_abs"]
    for w in range(len(om)):
        assert_points_match(np.concatenate([xg[w], yg[w]]), np.concatenate([xo[w], yo[w]]),
                            1e-10, f"weight {w}")
        np.testing.assert_allclose([kk[w][k] for k in keys], parts[w], rtol=1e-9, atol=1e-12)
    assert best == obest
