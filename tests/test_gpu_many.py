"""pdhg_solve_many: several independent LPs solved at once, the ones on the
one-workgroup path in shared launches (one workgroup per LP).  Every handle
must end exactly where its own pdhg_solve ends (same kernel, same checks):
iteration count, restarts, converged point, and bitwise equal iterates.
"""
import ctypes as C
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


def _lps():
    return [
        lpgen.small_dense(1), lpgen.small_dense(2), lpgen.small_dense(3),
        lpgen.bernoulli_lp(11, 30, 60, 0.15, lpgen.BOX01, ge_frac=0.4),
        lpgen.column_count_lp(13, 120, 260, per_col=3, bounds="mixed_inf", ge_frac=0.5),
        lpgen.bernoulli_lp(21, 40, 90, 0.5, lpgen.BOX01),            # other lane counts
        lpgen.column_count_lp(27, 300, 724, per_col=2, bounds="mix", ge_frac=0.3),  # matrix in LDS
        lpgen.column_count_lp(3, 3000, 7000, counts="powerlaw2", values="loguniform",
                              bounds="mix"),                         # multi-kernel path
    ]


def _solvers(lib, lps, **kw):
    return [lib.Solver(lp, eta=0.9 / _sigma_bound(lp), **kw) for lp in lps]


def _sigma_bound(lp):
    A = abs(lp.scipy_csr())
    return float(np.sqrt(float(A.sum(axis=0).max()) * float(A.sum(axis=1).max())))


def _same_state(a, b):
    for which in (0, 1, 2):
        xa, ya = a.get_iterate(which)
        xb, yb = b.get_iterate(which)
        torch.cuda.synchronize()
        assert torch.equal(xa, xb) and torch.equal(ya, yb), which
    ia, ib = a.info(), b.info()
    for key in ("k", "t", "restarts", "checks", "rho_prev"):
        assert ia[key] == ib[key], key


@pytest.mark.parametrize("budget,tol", [(400_000, 1e-8), (3_017, 0.0), (1_000, 1e-8)])
def test_solve_many_matches_single_solves(lib, budget, tol):
    lps = _lps()
    paths = [s.info()["one_workgroup"] for s in _solvers(lib, lps)]
    assert paths.count(0) == 1 and 2 in paths and (1 in paths or 3 in paths)
    _say("many", budget, tol)
    single = _solvers(lib, lps)
    ref = [s.solve(budget, tol) for s in single]
    many = _solvers(lib, lps)
    got = lib.solve_many(many, budget, tol)
    for i, (r, g) in enumerate(zip(ref, got)):
        assert g == r, (i, g, r)
        _same_state(single[i], many[i])


def test_solve_many_mid_block_start_and_mixed_methods(lib):
    """Handles that start between check points, and an extragradient handle
    (not on the one-workgroup path), next to plain ones."""
    lps = _lps()[:5]
    single = _solvers(lib, lps)
    many = _solvers(lib, lps)
    for s in single + many:
        s.step(7)
    egm = [lib.Solver(lps[0], eta=0.9 / _sigma_bound(lps[0]), method=lib.METHOD_EGM)
           for _ in range(2)]
    ref = [s.solve(20_000, 1e-8) for s in single + egm[:1]]
    got = lib.solve_many(many + egm[1:], 20_000, 1e-8)
    for i, (r, g) in enumerate(zip(ref, got)):
        assert g == r, (i, g, r)
    for a, b in zip(single + egm[:1], many + egm[1:]):
        _same_state(a, b)


def test_solve_many_continues_and_rejects_bad_arguments(lib):
    lps = _lps()[:3]
    single = _solvers(lib, lps)
    many = _solvers(lib, lps)
    for _ in range(2):  # a second call continues from where the first stopped
        ref = [s.solve(2_000, 0.0) for s in single]
        got = lib.solve_many(many, 2_000, 0.0)
        assert got == ref
    for a, b in zip(single, many):
        _same_state(a, b)
    L = lib.load(build_if_missing=False)
    hs = (C.c_void_p * 2)(many[0].h, many[0].h)
    need = int(L.pdhg_solve_many_workspace_bytes(2))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    res = (lib.Result * 2)()
    rc = L.pdhg_solve_many(C.cast(hs, C.c_void_p), 2, 10, 0.0, ws.data_ptr(), need,
                           C.cast(res, C.c_void_p))
    assert rc == lib.E_INVALID  # the same handle twice
    hs = (C.c_void_p * 2)(many[0].h, many[1].h)
    rc = L.pdhg_solve_many(C.cast(hs, C.c_void_p), 2, 10, 0.0, ws.data_ptr(), need - 1,
                           C.cast(res, C.c_void_p))
    assert rc == lib.E_INVALID  # workspace too small
    assert lib.solve_many([], 10, 0.0) == []


def test_solve_many_more_lps_than_compute_units(lib):
    """300 handles (more workgroups than the chip's 256 CUs), a third of them
    already converged before the call."""
    lp = lpgen.bernoulli_lp(11, 30, 60, 0.15, lpgen.BOX01, ge_frac=0.4)
    eta = 0.9 / _sigma_bound(lp)
    ref = lib.Solver(lp, eta=eta)
    r_ref = ref.solve(100_000, 1e-8)
    handles = [lib.Solver(lp, eta=eta) for _ in range(300)]
    for s in handles[::3]:
        s.solve(100_000, 1e-8)
    got = lib.solve_many(handles, 100_000, 1e-8)
    for i, g in enumerate(got):
        assert g["status"] == 0
        if i % 3:
            assert g == r_ref, i
    _same_state(ref, handles[1])
    _same_state(ref, handles[299])
