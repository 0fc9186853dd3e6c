"""Checkpoint and resume of Algorithm 1's state, and the failure outcomes of
the C ABI, on the GPU.

Checkpoint: a run stopped in the middle of an averaging window (k = 47,
t = 17 after the restart at the first check) and resumed from
pdhg_get_state / pdhg_set_state in a fresh handle follows the uninterrupted
run bit for bit to k = 1000 (iterates, averages, anchors, counters, check
log), and both follow the oracle (tolerance of tests/parity.py).

Failures, each forced from host data so that every kernel exits normally:
  - a step size far above 1/sigma_max(A) on an LP with free variables makes
    the iterates overflow: pdhg_solve and pdhg_restart_check return
    PDHG_E_NUMERICAL (the oracle's iterates overflow at the same point);
  - an infeasible LP: pdhg_solve returns PDHG_NOT_CONVERGED at the
    iteration budget, like the oracle;
  - a workspace one byte short, misaligned or missing: pdhg_create returns
    PDHG_E_WORKSPACE;
  - a state of another LP or another configuration: PDHG_E_INVALID.
"""
import ctypes as C
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2105_12715_amd import lpgen
from tests.lp_cases import lp_from_dense
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


def _solver(lib, lp, tiny_off=False, **kw):
    if tiny_off:
        os.environ["PDHG_TINY"] = "0"
    try:
        return lib.Solver(lp, **kw)
    finally:
        os.environ.pop("PDHG_TINY", None)


def _points(s, lib):
    out = []
    for which in (0, 1, 2, 3):
        x, y = s.get_iterate(which)
        out.append((x.clone(), y.clone()))
    torch.cuda.synchronize()
    return out


CASES = {
    # multi-kernel path, >= rows and infinite bounds of every kind
    "mixed_inf": (lambda: lpgen.column_count_lp(13, 600, 1300, per_col=5, bounds="mixed_inf",
                                                ge_frac=0.5), False),
    # one-workgroup path
    "small50x100": (lambda: lpgen.small_dense(1), False),
    # the same small LP forced onto the multi-kernel path
    "small_multi": (lambda: lpgen.small_dense(1), True),
}


@pytest.mark.parametrize("mode,method", [(oracle.MODE_ADAPTIVE, oracle.METHOD_PDHG),
                                         (oracle.MODE_FLEXIBLE, oracle.METHOD_PDHG),
                                         (oracle.MODE_FIXED, oracle.METHOD_PDHG),
                                         (oracle.MODE_ADAPTIVE, oracle.METHOD_EGM)])
@pytest.mark.parametrize("case", list(CASES))
def test_resume_mid_window_is_bitwise(lib, case, mode, method):
    make, tiny_off = CASES[case]
    lp = make()
    eta = oracle.Oracle(lp).info()["eta"]
    kw = dict(restart_mode=mode, fixed_len=40, method=method)
    _say("resume", case, mode, method)
    a = _solver(lib, lp, tiny_off, eta=eta, **kw)
    a.solve(47, 0.0)
    info = a.info()
    assert info["k"] == 47
    if mode != oracle.MODE_FIXED:
        assert info["t"] == 17 and info["restarts"] == 1
    st = a.get_state()
    # a fresh handle created with the step size of its own power iteration:
    # the state brings the step size of the run it was taken from
    b = _solver(lib, lp, tiny_off, **kw)
    b.set_state(st)
    assert b.info()["eta"] == info["eta"]
    for key in ("k", "t", "restarts", "checks", "rho_prev"):
        assert b.info()[key] == info[key], key
    # the uninterrupted run and the resumed one, and the oracle beside them
    o = oracle.Oracle(lp, eta=eta, mode=mode, fixed_len=40, method=method)
    o.solve(47, 0.0)
    for budget in (13, 940):
        a.solve(budget, 0.0)
        b.solve(budget, 0.0)
        o.solve(budget, 0.0)
    pa, pb = _points(a, lib), _points(b, lib)
    for (xa, ya), (xb, yb) in zip(pa, pb):
        assert torch.equal(xa, xb) and torch.equal(ya, yb)
    ia, ib = a.info(), b.info()
    for key in ("k", "t", "restarts", "checks", "rho_prev"):
        assert ia[key] == ib[key], key
    assert ia["k"] == 1000
    np.testing.assert_array_equal(a.check_log(), b.check_log())
    for which in (0, 1, 2):
        xo, yo = o.get(which)
        xg, yg = (t.cpu().numpy() for t in pa[which])
        assert_points_match(np.concatenate([xg, yg]), np.concatenate([xo, yo]), 1e-10,
                            f"point {which}")
    assert ia["restarts"] == o.info()["restarts"]


def test_resume_after_converged_solve_returns_same_solution(lib):
    lp = lpgen.column_count_lp(13, 600, 1300, per_col=5, bounds="mixed_inf", ge_frac=0.5)
    eta = oracle.Oracle(lp).info()["eta"]
    a = lib.Solver(lp, eta=eta)
    ra = a.solve(400_000, 1e-8)
    assert ra["status"] == 0
    b = lib.Solver(lp, eta=eta)
    b.set_state(a.get_state())
    xa, ya = a.get_iterate(lib.POINT_SOLUTION)
    xb, yb = b.get_iterate(lib.POINT_SOLUTION)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb) and torch.equal(ya, yb)
    ia, ib = a.info(), b.info()
    assert (ia["k"], ia["restarts"], ia["checks"]) == (ib["k"], ib["restarts"], ib["checks"])
    assert ib["k"] == ra["k"]


def test_set_state_rejects_other_lp_or_configuration(lib):
    lp = lpgen.column_count_lp(13, 600, 1300, per_col=5, bounds="mixed_inf", ge_frac=0.5)
    a = lib.Solver(lp, eta=0.1)
    a.solve(60, 0.0)
    st = a.get_state()
    # same sizes, other matrix
    other = lpgen.column_count_lp(14, 600, 1300, per_col=5, bounds="mixed_inf", ge_frac=0.5)
    assert other.nnz == lp.nnz
    with pytest.raises(lib.PdhgError) as e:
        lib.Solver(other, eta=0.1).set_state(st)
    assert e.value.code == lib.E_INVALID
    # other sizes
    with pytest.raises(lib.PdhgError) as e:
        lib.Solver(lpgen.small_dense(1), eta=0.1).set_state(st)
    assert e.value.code in (lib.E_INVALID, lib.E_WORKSPACE)
    # other restart scheme
    with pytest.raises(lib.PdhgError) as e:
        lib.Solver(lp, eta=0.1, restart_mode=lib.RESTART_NONE).set_state(st)
    assert e.value.code == lib.E_INVALID
    # a buffer not written by pdhg_get_state
    b = lib.Solver(lp, eta=0.1)
    owner, view = st
    junk = torch.zeros_like(view)
    with pytest.raises(lib.PdhgError) as e:
        b.set_state((None, junk))
    assert e.value.code == lib.E_INVALID
    # too short
    rc = b._L.pdhg_set_state(b.h, C.c_void_p(view.data_ptr()), view.numel() - 1)
    assert rc == lib.E_WORKSPACE
    # the handle is unchanged after the errors
    b.solve(60, 0.0)
    xa, _ = a.get_iterate(0)
    xb, _ = b.get_iterate(0)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)


def _divergent_lp():
    rng = np.random.default_rng(0)
    k = 12
    s = rng.uniform(0.5, 2.0, k)
    A = -np.diag(s)
    A[0, 1] = 0.3
    A[3, 2] = -0.4
    lp = lp_from_dense(A, rng.standard_normal(k), rng.standard_normal(k), [-np.inf] * k,
                       [np.inf] * k)
    return lp, float(np.linalg.norm(A, 2))


@pytest.mark.parametrize("tiny_off", [False, True])
def test_step_size_too_large_is_a_numerical_error(lib, tiny_off):
    """eta = 3 / sigma_max(A) (the valid range is eta <= 1/sigma_max) on an
    LP whose variables are all free: the PDHG map expands, the iterates
    overflow, and the first check whose KKT sums are not finite (the
    oracle's KKT values overflow at the same check) ends the solve with
    PDHG_E_NUMERICAL."""
    lp, smax = _divergent_lp()
    eta = 3.0 / smax
    o = oracle.Oracle(lp, eta=eta)
    o.solve(600, 1e-8)
    lo = o.log()
    bad = [int(r[0]) for r in lo if not np.all(np.isfinite(r[3:5]))]
    assert bad, "the oracle's KKT values stay finite"
    k_bad = bad[0]  # the first check whose KKT sums overflow
    s = _solver(lib, lp, tiny_off, eta=eta)
    assert (s.info()["one_workgroup"] == 0) == tiny_off
    with pytest.raises(lib.PdhgError) as e:
        s.solve(6000, 1e-8)
    assert e.value.code == lib.E_NUMERICAL
    # the run stops at the check that saw the breakdown
    assert s.info()["k"] == k_bad
    lg = s.check_log()
    np.testing.assert_array_equal(lg[:, 0], lo[: lg.shape[0], 0])
    # the handle stays usable and keeps reporting the breakdown
    s.step(30)
    with pytest.raises(lib.PdhgError) as e:
        s.check(1e-8)
    assert e.value.code == lib.E_NUMERICAL


@pytest.mark.parametrize("tiny_off", [False, True])
def test_infeasible_lp_is_not_converged_at_budget(lib, tiny_off):
    """x1 + x2 = 5 with 0 <= x <= 1 has no solution: the solve uses its
    whole budget and reports PDHG_NOT_CONVERGED, as the oracle does."""
    lp = lp_from_dense(np.array([[1.0, 1.0]]), [5.0], [1.0, 1.0], [0, 0], [1, 1])
    o = oracle.Oracle(lp)
    ro = o.solve(3000, 1e-8)
    assert ro["status"] == 1 and ro["k"] == 3000
    s = _solver(lib, lp, tiny_off, eta=o.info()["eta"])
    rg = s.solve(3000, 1e-8)
    assert rg["status"] == lib.NOT_CONVERGED and rg["k"] == 3000
    assert rg["restarts"] == ro["restarts"]
    assert rg["kkt"] == pytest.approx(ro["kkt"], rel=1e-9)


def test_workspace_too_small_or_misaligned(lib):
    lp = lpgen.small_dense(2)
    s = lib.Solver(lp, eta=0.1)  # owns device copies of the LP in the API layout
    L = s._L
    need = L.pdhg_workspace_bytes(lp.m, lp.n, lp.nnz)
    owner, ws = lib._dev_workspace(need + 512, s.device)
    h = C.c_void_p()
    base = ws.data_ptr()
    stream = lib._stream_handle(None)
    rc = L.pdhg_create(C.byref(s._lp), C.byref(s.params), C.c_void_p(base), need - 1, stream,
                       C.byref(h))
    assert rc == lib.E_WORKSPACE and not h.value
    rc = L.pdhg_create(C.byref(s._lp), C.byref(s.params), C.c_void_p(base + 8), need, stream,
                       C.byref(h))
    assert rc == lib.E_WORKSPACE and not h.value
    rc = L.pdhg_create(C.byref(s._lp), C.byref(s.params), None, need, stream, C.byref(h))
    assert rc == lib.E_WORKSPACE and not h.value
    rc = L.pdhg_create(C.byref(s._lp), C.byref(s.params), C.c_void_p(base), need, stream,
                       C.byref(h))
    assert rc == lib.OK and h.value
    L.pdhg_destroy(h)
