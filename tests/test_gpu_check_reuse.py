"""The first primal half-step after a check takes the check's A'y instead of
running the product (the check computes A'y of the current y and A'y-bar
for its KKT sums; after a restart at the average, y is y-bar).  The check's
products run the same launches as the primal half-step's, so the update
must be bitwise the one with the product: iterates, running sums, counters
and check records equal bit for bit against PDHG_CHECK_REUSE=0, over solves
that start on and off the check period, with restarts at the average and
(flexible restarts) at the current point, with column slabs of y, and
across the calls that change the state or the product layout between
solves.
"""
import os
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


CASES = {
    # multi-kernel path (too large for one workgroup), power-law columns
    "powerlaw": (lambda: lpgen.column_count_lp(3, 3000, 7000, counts="powerlaw2",
                                               values="loguniform", bounds="mix"), None),
    # the medium LP with A'y over two column slabs of y
    "medium_slabs": (lambda: lpgen.medium(2), "65536"),
}


def _make(lib, lp, env, reuse, **kw):
    saved = {k: os.environ.get(k) for k in ("PDHG_CHECK_REUSE", "PDHG_SLAB_BYTES", "PDHG_TINY")}
    os.environ["PDHG_TINY"] = "0"
    if env:
        os.environ["PDHG_SLAB_BYTES"] = env
    if not reuse:
        os.environ["PDHG_CHECK_REUSE"] = "0"
    try:
        return lib.Solver(lp, **kw)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _same(a, b, where):
    for which in (0, 1, 2):
        xa, ya = a.get_iterate(which)
        xb, yb = b.get_iterate(which)
        torch.cuda.synchronize()
        assert torch.equal(xa, xb) and torch.equal(ya, yb), (where, which)
    ia, ib = a.info(), b.info()
    for key in ("k", "t", "restarts", "checks", "rho_prev"):
        assert ia[key] == ib[key], (where, key)
    np.testing.assert_array_equal(a.check_log(), b.check_log(), err_msg=where)


@pytest.mark.parametrize("mode", ["adaptive", "flexible"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_check_reuse_is_bitwise(lib, name, mode):
    mk, slab = CASES[name]
    lp = mk()
    rm = lib.RESTART_ADAPTIVE if mode == "adaptive" else lib.RESTART_FLEXIBLE
    a = _make(lib, lp, slab, True, restart_mode=rm)
    b = _make(lib, lp, slab, False, restart_mode=rm, eta=a.info()["eta"])
    assert a.info()["one_workgroup"] == 0
    _say("reuse", name, mode)
    done = 0
    for k in (30, 61, 300, 1200, 3000):
        a.solve(k - done, 0.0)
        b.solve(k - done, 0.0)
        done = k
        _same(a, b, f"{name} {mode} k={k}")
    assert a.info()["restarts"] >= 1
    # eager steps and checks between solves, then solves again
    for s in (a, b):
        s.step(7)
        s.check(0.0)
        s.solve(23 + 300, 0.0)
    _same(a, b, f"{name} {mode} after eager steps")
    # a new point: the next block must run its product again
    x, y = a.get_iterate(0)
    x2, y2 = x * 0.5, y * 0.5
    for s in (a, b):
        s.set_iterate(x2, y2)
        s.solve(600, 0.0)
    _same(a, b, f"{name} {mode} after set_iterate")
    # to tolerance
    ra = a.solve(200_000, 1e-8)
    rb = b.solve(200_000, 1e-8)
    assert ra == rb
    _same(a, b, f"{name} {mode} solved")


def test_check_reuse_after_layout_changes(lib):
    """A new SpMV layout (column slabs, lanes per row) sums A'y in another
    order, so the block after the change must run its product again rather
    than take the check's A'y from the old layout: bitwise equal to a solver
    that never reuses it, through two layout changes."""
    lp = lpgen.medium(2)
    a = _make(lib, lp, "65536", True)
    b = _make(lib, lp, "65536", False, eta=a.info()["eta"])
    for s in (a, b):
        s.solve(600, 0.0)
    _same(a, b, "before the changes")
    for sched in ((1, 1, 0, 0), (2, 2, 0, 1)):
        for s in (a, b):
            s.set_schedule(*sched)
            s.solve(630, 0.0)
        _same(a, b, f"schedule {sched}")


def test_batch_check_reuse_is_bitwise(lib):
    """The batched solver takes the check's A'y the same way: per LP, A'y, or
    A'y-bar when that LP restarted at its average; blocks of one converged LP
    do nothing and blocks of several LPs update every row (a converged LP's
    with step 0), as the product's launch does.  Small LPs converge early and
    share blocks of A' with each other and with the larger members, so the
    later solves run over converged LPs too; every iterate stays bitwise equal
    to the batch that never reuses the check's products."""
    lps = [lpgen.small_dense(5), lpgen.batch_member(2), lpgen.small_dense(6),
           lpgen.small_dense(7), lpgen.batch_member(3), lpgen.small_dense(8)]
    import oracle
    params = [{"eta": oracle.Oracle(lp).info()["eta"]} for lp in lps]
    saved = os.environ.get("PDHG_CHECK_REUSE")
    a = lib.BatchSolver(lps, params=params)
    os.environ["PDHG_CHECK_REUSE"] = "0"
    try:
        b = lib.BatchSolver(lps, params=params)
    finally:
        if saved is None:
            os.environ.pop("PDHG_CHECK_REUSE", None)
        else:
            os.environ["PDHG_CHECK_REUSE"] = saved

    def same(where):
        for i in range(len(lps)):
            for w in (0, 1, 2):
                xa, ya = a.get_iterate(i, w)
                xb, yb = b.get_iterate(i, w)
                assert torch.equal(xa, xb) and torch.equal(ya, yb), (where, i, w)
            ia, ib = a.info(i), b.info(i)
            for key in ("k", "t", "restarts", "checks"):
                assert ia[key] == ib[key], (where, i, key)

    for s in (a, b):
        s.solve(331, 0.0)
    same("331 iterations")
    ra = a.solve(30_000, 1e-8)
    rb = b.solve(30_000, 1e-8)
    assert ra == rb
    done = [r["status"] == 0 for r in ra]
    assert any(done) and not all(done)
    same("some converged")
    for s in (a, b):
        s.step(11)
        s.solve(3_019, 1e-8)
    same("after eager steps, over converged LPs")
