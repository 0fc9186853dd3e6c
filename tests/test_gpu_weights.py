"""GPU parity of the primal-weight search (Section 7) and of setting the
weight, through the C ABI, against the oracle's independent runs.

Every copy's last iterate matches its own oracle run to a relative 1e-10,
the KKT parts to 1e-9 relative, and the chosen weight exactly.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2105_12715_amd import lpgen
from tests.parity import assert_points_match

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PAPER_WEIGHTS = [4.0 ** k for k in range(-5, 6)]


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

KEYS = ["kkt_rel", "primal_res", "dual_res", "pobj", "dobj", "kkt_paper_abs", "kkt_max_abs"]


def _compare(lp, omegas, iters, s, eta):
    kk, best, xg, yg = s.weight_search(omegas, iters, want_iterates=True)
    parts, obest, xo, yo = oracle.weight_search(lp, omegas, iters, eta)
    xg, yg = xg.cpu().numpy(), yg.cpu().numpy()
    for w in range(len(omegas)):
        zg = np.concatenate([xg[w], yg[w]])
        zo = np.concatenate([xo[w], yo[w]])
        assert_points_match(zg, zo, 1e-10, f"weight {w}")
        got = [kk[w][k] for k in KEYS]
        np.testing.assert_allclose(got, parts[w], rtol=1e-9, atol=1e-12)
        assert kk[w]["kkt"] == kk[w]["kkt_paper_abs"]
    assert best == obest
    return best


@pytest.mark.parametrize("name,iters", [("small50x100", 300), ("ge_rows", 73),
                                        ("mixed_inf", 300), ("powerlaw", 150)])
def test_weight_search_matches_oracle(lib, name, iters):
    lp = CASES[name]()
    _say("weight search", name, iters)
    eta = oracle.Oracle(lp).info()["eta"]
    s = lib.Solver(lp, eta=eta)
    _compare(lp, PAPER_WEIGHTS, iters, s, eta)


def test_paper_search_on_a_table2_shaped_lp(lib):
    """The paper's search: 11 weights 4^-5..4^5, 5000 iterations, on a
    planted LP with the size of qap10 in Table 2 (1820 x 4150, 18200
    entries)."""
    lp = lpgen.paper_shaped("qap10")
    _say("weight search qap10-shaped", lp.m, lp.n, lp.nnz)
    eta = oracle.Oracle(lp).info()["eta"]
    s = lib.Solver(lp, eta=eta)
    _compare(lp, PAPER_WEIGHTS, 5000, s, eta)


def test_set_primal_weight_restarts_from_the_initial_point(lib):
    lp = CASES["mixed_inf"]()
    _say("set primal weight")
    eta = oracle.Oracle(lp).info()["eta"]
    s = lib.Solver(lp, eta=eta)
    s.solve(90, 0.0)
    s.set_primal_weight(4.0)
    info = s.info()
    assert info["k"] == 0 and info["restarts"] == 0 and info["checks"] == 0
    assert info["tau"] == eta / 4.0 and info["sigma"] == eta * 4.0
    o = oracle.Oracle(lp, eta=eta, omega=4.0)
    for k in (30, 300):
        o.solve(k - (30 if k == 300 else 0), 0.0)
        s.solve(k - (30 if k == 300 else 0), 0.0)
        for which in (0, 1, 2):
            xo, yo = o.get(which)
            xg, yg = (t.cpu().numpy() for t in s.get_iterate(which))
            assert_points_match(np.concatenate([xg, yg]), np.concatenate([xo, yo]), 1e-10,
                                f"point {which}")
    lo, lg = o.log(), s.check_log()
    assert lo.shape == lg.shape
    np.testing.assert_array_equal(lg[:, [0, 1, 2, 9, 10, 11]], lo[:, [0, 1, 2, 9, 10, 11]])


def test_weight_search_leaves_the_handle_alone(lib):
    lp = CASES["small50x100"]()
    s = lib.Solver(lp)
    s.solve(60, 0.0)
    x0, y0 = (t.clone() for t in s.get_iterate(0))
    k0 = s.info()["k"]
    s.weight_search([0.5, 2.0], 100)
    x1, y1 = s.get_iterate(0)
    assert torch.equal(x0, x1) and torch.equal(y0, y1) and s.info()["k"] == k0


def test_weight_search_rejects_bad_arguments(lib):
    lp = CASES["small50x100"]()
    s = lib.Solver(lp)
    for om in ([], [1.0] * 17, [1.0, 0.0], [1.0, -2.0], [np.nan], [np.inf]):
        with pytest.raises((lib.PdhgError, ValueError)):
            s.weight_search(om, 10)
    with pytest.raises(lib.PdhgError):
        s.weight_search([1.0], -1)
    for om in (0.0, -1.0, np.nan, np.inf):
        with pytest.raises(lib.PdhgError):
            s.set_primal_weight(om)
