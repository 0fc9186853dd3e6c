"""Pins for the oracle's KKT error, restart logic, power iteration,
transpose and whole solves."""
import itertools
import json
import os

import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from paper_2105_12715_amd import lpgen
from tests.lp_cases import dense_A, lp_from_dense, planted_cases

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ KKT ---

def test_kkt_hand_worked_2x3():
    g = json.load(open(os.path.join(GOLD, "kkt_2x3.json")))
    u = [np.inf if v == "inf" else v for v in g["u"]]
    lp = lp_from_dense(g["A"], g["b"], g["c"], g["l"], u, g["row_kind"])
    o = oracle.Oracle(lp, eta=0.1)
    for pt in g["points"]:
        out = o.kkt_at(np.array(pt["x"], float), np.array(pt["y"], float))
        assert out[0] == pytest.approx(pt["kkt_rel"], rel=1e-14)
        assert out[1] == pytest.approx(pt["primal_res"], abs=1e-15)
        assert out[2] == pytest.approx(pt["dual_res"], abs=1e-15)
        assert out[3] == pytest.approx(pt["pobj"], rel=1e-15)
        assert out[4] == pytest.approx(pt["dobj"], rel=1e-15)
        assert out[5] == pytest.approx(pt["kkt_paper_abs"], rel=1e-14)
        assert out[6] == pytest.approx(pt["kkt_max_abs"], rel=1e-15)


@pytest.mark.parametrize("case", range(6))
def test_kkt_zero_at_planted_optimum(case):
    lp = planted_cases()[case]
    o = oracle.Oracle(lp, eta=0.1)
    out = o.kkt_at(lp.x_star, lp.y_star)
    assert out[0] <= 1e-14
    assert out[5] <= 1e-12 * (1 + np.abs(lp.c).sum())


@pytest.mark.parametrize("seed", range(5))
def test_kkt_paper_abs_equals_K_h_matrix_form(seed):
    """Standard form: the paper-abs KKT equals ||(h - Kz)^+||_2 with K and h
    assembled as matrices from eq. define:K-and-h-for-lp."""
    rng = np.random.default_rng(seed)
    m, n = 5, 8
    A = rng.standard_normal((m, n)) * (rng.random((m, n)) < 0.6)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    lp = lp_from_dense(A, b, c, [0.0] * n, [np.inf] * n)
    o = oracle.Oracle(lp, eta=0.1)
    K = np.block([
        [np.eye(n), np.zeros((n, m))],
        [-A, np.zeros((m, m))],
        [A, np.zeros((m, m))],
        [np.zeros((n, n)), -A.T],
        [-c[None, :], b[None, :]],
    ])
    h = np.concatenate([np.zeros(n), -b, b, -c, [0.0]])
    for _ in range(5):
        x = rng.standard_normal(n)
        y = rng.standard_normal(m)
        z = np.concatenate([x, y])
        ref = np.linalg.norm(np.maximum(h - K @ z, 0.0))
        # the A x = b block appears twice in K (>= and <=); only one side
        # of each pair is violated, so the norm is unchanged
        assert o.kkt_at(x, y)[5] == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("seed", range(4))
def test_weak_duality_of_dual_objective(seed):
    """For y with y >= 0 on >= rows the dual objective is a lower bound on
    c'x for every feasible x; in particular dobj(y) <= c'x*."""
    lp = planted_cases()[seed + 2]
    o = oracle.Oracle(lp, eta=0.1)
    rng = np.random.default_rng(seed)
    for _ in range(20):
        y = lp.y_star + rng.standard_normal(lp.m)
        y[lp.row_kind == 1] = np.abs(y[lp.row_kind == 1])
        out = o.kkt_at(lp.x_star, y)
        if out[2] == 0.0:  # dual residual zero: a dual-feasible y
            assert out[4] <= lp.objective_star() + 1e-9
        else:
            # a bound is missing where the reduced cost points; the dual
            # objective then ignores that coordinate and the residual is > 0
            assert out[2] > 0.0


# ------------------------------------------------------- restart logic ---

@pytest.mark.parametrize("mode", [oracle.MODE_ADAPTIVE, oracle.MODE_FLEXIBLE])
def test_adaptive_restart_decisions_follow_the_rule(mode):
    """eq. adaptive-restart-scheme with tau^0 = 1 and beta = 1/e: the first
    check restarts; later ones restart iff rho(candidate) <= beta rho_prev,
    and rho_prev is the candidate's rho at the previous restart."""
    lp = planted_cases()[0]
    o = oracle.Oracle(lp, mode=mode)
    o.solve(3000, 0.0)
    log = o.log()
    assert log.shape[0] == 100
    beta = np.exp(-1.0)
    rho_prev = None
    n_rst = 0
    for rec in log:
        rho_a = rec[6]
        cand = rho_a
        if mode == oracle.MODE_FLEXIBLE and rec[8] < rho_a:
            cand = rec[8]
            assert rec[10] == 1
        else:
            assert rec[10] == 0
        assert rec[2] == n_rst
        if n_rst == 0:
            expect = True
        else:
            assert rec[12] == rho_prev
            expect = cand <= beta * rho_prev
        assert bool(rec[9]) == expect
        if expect:
            n_rst += 1
            rho_prev = cand
    assert n_rst >= 3


def test_restart_anchor_radius_and_window():
    lp = planted_cases()[1]
    o = oracle.Oracle(lp, mode=oracle.MODE_ADAPTIVE)
    o.solve(30, 0.0)  # first check restarts unconditionally (tau^0 = 1)
    info = o.info()
    assert info["restarts"] == 1 and info["t"] == 0
    x, y = o.get(0)
    x0, y0 = o.get(2)
    np.testing.assert_array_equal(x, x0)
    o.step(30)
    xa, ya = o.get(1)
    rho, r, _ = o.gap(1)
    assert r == pytest.approx(np.sqrt(np.sum((xa - x0) ** 2) + np.sum((ya - y0) ** 2)), rel=1e-14)


@pytest.mark.parametrize("mode", [oracle.MODE_ADAPTIVE, oracle.MODE_FLEXIBLE])
def test_restart_anchors_approach_optimum(mode):
    """Proposition thm:pdhg-ppm:bound-adaptive-restart-scheme: the distance
    of the restart anchors to z* never grows (PDHG norm)."""
    lp = planted_cases()[0]
    A = dense_A(lp)
    o = oracle.Oracle(lp, mode=mode)
    inf = o.info()

    def dist(x, y):
        dx, dy = x - lp.x_star, y - lp.y_star
        return dx @ dx / inf["tau"] + 2 * dy @ (A @ dx) + dy @ dy / inf["sigma"]

    prev = dist(*o.get(2))
    seen = 0
    for _ in range(200):
        o.solve(30, 0.0)
        if o.info()["restarts"] > seen:
            seen = o.info()["restarts"]
            d = dist(*o.get(2))
            assert d <= prev * (1 + 1e-10) + 1e-14
            prev = d
    assert seen >= 5


def test_fixed_length_restarts_every_T():
    lp = planted_cases()[2]
    o = oracle.Oracle(lp, mode=oracle.MODE_FIXED, fixed_len=64)
    for k in range(1, 300):
        o.step(1)
        assert o.info()["restarts"] == k // 64
        assert o.info()["t"] == k % 64


def test_no_restart_mode_never_restarts():
    lp = planted_cases()[2]
    o = oracle.Oracle(lp, mode=oracle.MODE_NONE)
    o.solve(900, 0.0)
    assert o.info()["restarts"] == 0 and o.info()["t"] == 900


# ----------------------------------------------------- power, transpose ---

@pytest.mark.parametrize("case", range(6))
def test_power_iteration_sigma_max(case):
    lp = planted_cases()[case]
    s = np.linalg.svd(dense_A(lp), compute_uv=False)[0]
    est = oracle.power_iteration(lp, 5000, 1e-14)
    assert est == pytest.approx(s, rel=1e-6)
    assert est <= s * (1 + 1e-12)
    o = oracle.Oracle(lp)
    inf = o.info()
    assert inf["eta"] == pytest.approx(0.9 / inf["sigma_max"], rel=1e-15)
    assert inf["eta"] * s < 1.0


def test_transpose_matches_scipy():
    lp = lpgen.column_count_lp(3, 300, 700, counts="powerlaw2")
    trp, tci, tv, perm = oracle.transpose(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.vals)
    At = lp.scipy_csr().T.tocsr()
    At.sort_indices()
    np.testing.assert_array_equal(trp, At.indptr)
    np.testing.assert_array_equal(tci, At.indices)
    np.testing.assert_array_equal(tv, At.data)
    np.testing.assert_array_equal(lp.vals[perm], tv)


# --------------------------------------------------------- whole solve ---

def _vertex_optimum(A, b, c, l, u):
    """Brute force over all bases: nonbasic variables sit at a bound, basic
    ones solve A_B x_B = b - A_N x_N; keep the feasible vertex of least cost."""
    m, n = A.shape
    best = np.inf
    for B in itertools.combinations(range(n), m):
        AB = A[:, B]
        if abs(np.linalg.det(AB)) < 1e-10:
            continue
        N = [j for j in range(n) if j not in B]
        for bits in itertools.product([0, 1], repeat=len(N)):
            xN = np.array([u[j] if t else l[j] for j, t in zip(N, bits)])
            if np.any(~np.isfinite(xN)):
                continue
            xB = np.linalg.solve(AB, b - A[:, N] @ xN)
            if np.all(xB >= l[list(B)] - 1e-9) and np.all(xB <= u[list(B)] + 1e-9):
                x = np.zeros(n)
                x[list(B)] = xB
                x[N] = xN
                best = min(best, c @ x)
    return best


@pytest.mark.parametrize("seed", range(8))
def test_solve_matches_vertex_enumeration(seed):
    lp = lpgen.bernoulli_lp(200 + seed, 3, 7, 0.7, lpgen.BOX01)
    A = dense_A(lp)
    if np.linalg.matrix_rank(A) < lp.m:
        pytest.skip("rank-deficient draw")
    ref = _vertex_optimum(A, lp.b, lp.c, lp.l, lp.u)
    o = oracle.Oracle(lp, mode=oracle.MODE_ADAPTIVE)
    res = o.solve(200000, 1e-10)
    assert res["status"] == 0
    assert res["pobj"] == pytest.approx(ref, rel=1e-7, abs=1e-8)
    assert ref == pytest.approx(lp.objective_star(), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("case", range(6))
def test_solve_matches_highs(case):
    lp = planted_cases()[case]
    A = lp.scipy_csr()
    eq = lp.row_kind == 0
    bounds = [(None if np.isinf(a) else a, None if np.isinf(b_) else b_)
              for a, b_ in zip(lp.l, lp.u)]
    kw = {}
    if eq.any():
        kw.update(A_eq=A[eq], b_eq=lp.b[eq])
    if (~eq).any():
        kw.update(A_ub=-A[~eq], b_ub=-lp.b[~eq])
    ref = linprog(lp.c, bounds=bounds, method="highs", **kw)
    assert ref.status == 0
    o = oracle.Oracle(lp, mode=oracle.MODE_ADAPTIVE)
    res = o.solve(400000, 1e-9)
    assert res["status"] == 0
    scale = 1 + abs(ref.fun)
    assert abs(res["pobj"] - ref.fun) <= 1e-6 * scale
    assert abs(res["pobj"] - lp.objective_star()) <= 1e-6 * scale
    # strong duality at the returned point
    assert abs(res["pobj"] - res["dobj"]) <= 1e-6 * scale


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_small_dense_reaches_1e8(seed):
    lp = lpgen.small_dense(seed)
    o = oracle.Oracle(lp, mode=oracle.MODE_ADAPTIVE)
    res = o.solve(200000, 1e-8)
    assert res["status"] == 0 and res["kkt"] <= 1e-8
    assert res["pobj"] == pytest.approx(lp.objective_star(), rel=1e-6)
    x = res["x"]
    assert np.all(x >= lp.l) and np.all(x <= lp.u)


def test_restarts_beat_no_restarts():
    """Table 3's qualitative pattern: without restarts PDHG stalls far above
    the accuracy the adaptive scheme reaches in the same iterations."""
    lp = lpgen.small_dense(1)
    a = oracle.Oracle(lp, mode=oracle.MODE_ADAPTIVE).solve(30000, 1e-8)
    n = oracle.Oracle(lp, mode=oracle.MODE_NONE).solve(30000, 1e-8)
    assert a["status"] == 0
    assert n["status"] == 1 and n["kkt"] > 100 * a["kkt"]
