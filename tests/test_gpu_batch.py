"""GPU parity of the batched solver: every LP of a batch follows its own
oracle run (same iterates to 1e-10, same check records, same iteration
count to 1e-8), whatever the other LPs in the batch do."""
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
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def batch_lps():
    return [
        lpgen.small_dense(1),
        lpgen.bernoulli_lp(11, 30, 60, 0.15, lpgen.BOX01, ge_frac=0.4),
        lpgen.column_count_lp(13, 600, 1300, per_col=5, bounds="mixed_inf", ge_frac=0.5),
        lpgen.column_count_lp(3, 3000, 7000, counts="powerlaw2", values="loguniform", bounds="mix"),
        lpgen.small_dense(4),
        lpgen.column_count_lp(21, 2500, 5000, per_col=5, bounds="box01"),
    ]


def _cmp(o, b, i, tol=1e-10):
    for which in (0, 1, 2):
        xo, yo = o.get(which)
        xg, yg = (t.cpu().numpy() for t in b.get_iterate(i, which))
        assert_points_match(np.concatenate([xg, yg]), np.concatenate([xo, yo]), tol,
                            f"LP {i} point {which}")


@pytest.mark.parametrize("mode", [1, 2])
def test_batch_iterates_and_logs_match_oracle(lib, mode):
    lps = batch_lps()
    _say("batch iterates mode", mode)
    etas = [oracle.Oracle(lp).info()["eta"] for lp in lps]
    orcs = [oracle.Oracle(lp, eta=e, mode=mode) for lp, e in zip(lps, etas)]
    b = lib.BatchSolver(lps, params=[{"eta": e} for e in etas], restart_mode=mode)
    assert b.info(0)["bound_classes"] == 0  # six (l, u) pairs in the mixed member
    done = 0
    for k in [30, 31, 90, 300, 1000]:
        b.solve(k - done, 0.0)
        for o in orcs:
            o.solve(k - done, 0.0)
        done = k
        for i, o in enumerate(orcs):
            _cmp(o, b, i)
    for i, o in enumerate(orcs):
        lo, lg = o.log(), b.check_log(i)
        assert lo.shape == lg.shape == (33, 14)
        np.testing.assert_array_equal(lg[:, [0, 1, 2, 9, 10, 11]], lo[:, [0, 1, 2, 9, 10, 11]])
        for col in (3, 4, 5, 6, 7, 8, 12):
            np.testing.assert_allclose(lg[:, col], lo[:, col], rtol=1e-9, atol=1e-300)


def test_batch_power_iteration_per_lp(lib):
    lps = batch_lps()
    _say("batch power iteration")
    b = lib.BatchSolver(lps)
    for i, lp in enumerate(lps):
        oi = oracle.Oracle(lp).info()
        gi = b.info(i)
        assert gi["sigma_max"] == pytest.approx(oi["sigma_max"], rel=1e-9)
        assert gi["eta"] == pytest.approx(0.9 / gi["sigma_max"], rel=1e-15)


def test_batch_solve_to_1e8_each_lp_like_its_oracle(lib):
    lps = batch_lps()[:3] + [lpgen.small_dense(7)]
    _say("batch solve")
    etas = [oracle.Oracle(lp).info()["eta"] for lp in lps]
    b = lib.BatchSolver(lps, params=[{"eta": e} for e in etas])
    res = b.solve(400_000, 1e-8)
    for i, (lp, e) in enumerate(zip(lps, etas)):
        ro = oracle.Oracle(lp, eta=e).solve(400_000, 1e-8)
        assert ro["status"] == 0 and res[i]["status"] == 0
        assert res[i]["k"] == ro["k"] and res[i]["restarts"] == ro["restarts"]
        assert res[i]["kkt"] <= 1e-8
        x, y = (t.cpu().numpy() for t in b.get_iterate(i, 3))
        assert oracle.Oracle(lp, eta=0.1).kkt_at(x, y)[0] <= 1.0001e-8


def test_batch_of_one_equals_single_solver(lib):
    lp = batch_lps()[2]
    _say("batch of one")
    eta = oracle.Oracle(lp).info()["eta"]
    b = lib.BatchSolver([lp], params=[{"eta": eta}])
    s = lib.Solver(lp, eta=eta)
    b.solve(600, 0.0)
    s.solve(600, 0.0)
    xb, yb = (t.cpu().numpy() for t in b.get_iterate(0))
    xs, ys = (t.cpu().numpy() for t in s.get_iterate(0))
    assert_points_match(np.concatenate([xb, yb]), np.concatenate([xs, ys]), 1e-12,
                        "batch member against its single solve")
    assert b.info(0)["restarts"] == s.info()["restarts"]


def test_uneven_batch_members(lib):
    """Members of the uneven batch workload (sizes drawn per LP)."""
    lps = [lpgen.batch_member(i) for i in range(4)]
    _say("uneven batch", [lp.m for lp in lps])
    etas = [oracle.Oracle(lp).info()["eta"] for lp in lps]
    orcs = [oracle.Oracle(lp, eta=e) for lp, e in zip(lps, etas)]
    b = lib.BatchSolver(lps, params=[{"eta": e} for e in etas])
    # one (l, u) pair over the batch: the primal update reads a class byte
    assert b.info(0)["bound_classes"] == 1
    b.solve(300, 0.0)
    for i, o in enumerate(orcs):
        o.solve(300, 0.0)
        _cmp(o, b, i)
    # runs of odd length (the running sums are updated in pairs of
    # iterations; an odd run ends with a single addition), then a solve that
    # starts between check points
    b.step(7)
    b.solve(53, 0.0)
    for i, o in enumerate(orcs):
        o.step(7)
        o.solve(53, 0.0)
        _cmp(o, b, i)


def test_member_wider_than_16_bit_indices(lib):
    """A member with more than 65,536 columns: the batch keeps 32-bit
    indices (smaller batches use 16-bit ones relative to each LP)."""
    lps = [lpgen.column_count_lp(31, 1200, 70_000, per_col=1, bounds="mix"),
           lpgen.small_dense(2)]
    _say("wide member", [(lp.m, lp.n) for lp in lps])
    etas = [oracle.Oracle(lp).info()["eta"] for lp in lps]
    orcs = [oracle.Oracle(lp, eta=e) for lp, e in zip(lps, etas)]
    b = lib.BatchSolver(lps, params=[{"eta": e} for e in etas])
    b.solve(301, 0.0)
    for i, o in enumerate(orcs):
        o.solve(301, 0.0)
        _cmp(o, b, i)


def test_members_without_rows_and_with_empty_columns(lib):
    """A member with no rows, one with empty columns and >= rows, and two
    ordinary ones: each SpMV block stays inside one member (a member
    without rows has only an empty block), columns are reordered inside
    each member, and every member follows its oracle."""
    from tests.lp_cases import lp_from_dense
    no_rows = lp_from_dense(np.zeros((0, 4)), [], [1.0, -1.0, 0.5, 0.0], [0, 0, -1, -2],
                            [1, 1, 1, 2])
    A = np.array([[1.0, 0, 2.0, 0], [0, 0, -1.0, 0], [3.0, 0, 0, 0]])
    empty_cols = lp_from_dense(A, [1.0, -0.5, 2.0], [1.0, 1.0, 1.0, -1.0], [0, 0, 0, -1],
                               [5, 5, 5, 3], kind=[0, 1, 0])
    lps = [lpgen.small_dense(3), no_rows, empty_cols,
           lpgen.column_count_lp(41, 900, 2000, per_col=3, bounds="mix", ge_frac=0.3)]
    _say("edge members", [(lp.m, lp.n) for lp in lps])
    etas = [0.5 if lp.m == 0 else oracle.Oracle(lp).info()["eta"] for lp in lps]
    orcs = [oracle.Oracle(lp, eta=e, mode=2) for lp, e in zip(lps, etas)]
    b = lib.BatchSolver(lps, params=[{"eta": e} for e in etas], restart_mode=2)
    done = 0
    for k in [1, 30, 61, 600]:
        b.solve(k - done, 0.0)
        for o in orcs:
            o.solve(k - done, 0.0)
        done = k
        for i, o in enumerate(orcs):
            _cmp(o, b, i)


def test_batch_paired_running_sums_are_exact(lib):
    """As for one LP: sixty one-iteration steps and one sixty-iteration step
    give bitwise the same iterates and averages."""
    lps = batch_lps()
    params = [{"eta": oracle.Oracle(lp).info()["eta"]} for lp in lps]
    a = lib.BatchSolver(lps, params=params, restart_mode=0)
    b = lib.BatchSolver(lps, params=params, restart_mode=0)
    for _ in range(60):
        a.step(1)
    b.step(60)
    for i in range(len(lps)):
        for which in (0, 1):
            xa, ya = a.get_iterate(i, which)
            xb, yb = b.get_iterate(i, which)
            torch.cuda.synchronize()
            assert torch.equal(xa, xb) and torch.equal(ya, yb), (i, which)


@pytest.mark.parametrize("placement,index16", [(1, 1), (1, 0), (0, 1), (0, 0)])
def test_batch_schedules_follow_the_oracle(lib, placement, index16):
    """Every SpMV schedule of the batch (XCD placement or row order; 16-bit
    or 32-bit indices) gives the oracle's iterates."""
    lps = [lpgen.batch_member(2), lpgen.batch_member(3), lpgen.small_dense(5),
           lpgen.column_count_lp(13, 600, 1300, per_col=5, bounds="mixed_inf", ge_frac=0.5)]
    etas = [oracle.Oracle(lp).info()["eta"] for lp in lps]
    orcs = [oracle.Oracle(lp, eta=e) for lp, e in zip(lps, etas)]
    b = lib.BatchSolver(lps, params=[{"eta": e} for e in etas])
    b.set_schedule(placement, index16)
    b.solve(307, 0.0)
    for i, o in enumerate(orcs):
        o.solve(307, 0.0)
        _cmp(o, b, i)


def test_batch_autotune(lib):
    """The tuner times the four schedules on products into scratch vectors:
    the iterates stay bitwise as they were, the fastest schedule is kept,
    and the solve goes on like the oracle's."""
    lps = [lpgen.batch_member(i) for i in range(4)]
    etas = [oracle.Oracle(lp).info()["eta"] for lp in lps]
    orcs = [oracle.Oracle(lp, eta=e) for lp, e in zip(lps, etas)]
    b = lib.BatchSolver(lps, params=[{"eta": e} for e in etas])
    b.solve(90, 0.0)
    before = [[t.clone() for t in b.get_iterate(i, w)] for i in range(4) for w in (0, 1)]
    r = b.autotune(5)
    _say("batch tune", r)
    after = [[t.clone() for t in b.get_iterate(i, w)] for i in range(4) for w in (0, 1)]
    for p, q in zip(before, after):
        assert torch.equal(p[0], q[0]) and torch.equal(p[1], q[1])
    assert len(r["ms"]) == 4
    assert min(r["ms"], key=r["ms"].get) == (r["placement"], r["index16"])
    b.solve(210, 0.0)
    for i, o in enumerate(orcs):
        o.solve(300, 0.0)
        _cmp(o, b, i)
    # 16-bit indices need every LP within 65,536 rows and columns
    wide = lib.BatchSolver([lpgen.column_count_lp(31, 1200, 70_000, per_col=1, bounds="mix")],
                           params=[{"eta": 0.01}])
    with pytest.raises(lib.PdhgError):
        wide.set_schedule(1, 1)
    wide.set_schedule(0, 0)
    assert len(wide.autotune(2)["ms"]) == 2


def test_batch_schedules_give_bitwise_equal_iterates(lib):
    """Placement and index width change which workgroup runs a block and how
    it addresses the gathered vector, not the order of any sum."""
    lps = [lpgen.batch_member(2), lpgen.small_dense(5), lpgen.batch_member(3)]
    params = [{"eta": oracle.Oracle(lp).info()["eta"]} for lp in lps]
    runs = []
    for placement, index16 in [(1, 1), (0, 0), (1, 0), (0, 1)]:
        b = lib.BatchSolver(lps, params=params)
        b.set_schedule(placement, index16)
        b.solve(331, 0.0)
        runs.append([[t.clone() for t in b.get_iterate(i, w)] for i in range(3) for w in (0, 1)])
    for other in runs[1:]:
        for p, q in zip(runs[0], other):
            assert torch.equal(p[0], q[0]) and torch.equal(p[1], q[1])
