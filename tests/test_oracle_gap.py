"""Pins for the oracle's linear trust region (Algorithm 2) and the
normalized duality gap rho_r(z) (eq. rhorz)."""
import os
import warnings

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from tests.lp_cases import dense_A, lp_from_dense, planted_cases

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def tr_sort_and_scan(a, d, r):
    """Independent exact solver: evaluate f(lambda) = sum min(lambda a, d)^2
    at every breakpoint directly, find the last breakpoint inside the ball
    and solve the quadratic on the following breakpoint-free interval."""
    a = np.asarray(a, float)
    d = np.asarray(d, float)
    act = a > 0
    a, d = a[act], d[act]
    if r <= 0:
        return 0.0
    if np.all(np.isfinite(d)) and np.sum(d * d) <= r * r:
        return float(np.sum(a * d))
    bp = d / a
    fin = np.unique(bp[np.isfinite(bp)])

    def f(lam):
        return np.sum(np.minimum(lam * a, d) ** 2)

    lam_k = 0.0
    for v in fin:
        if f(v) <= r * r:
            lam_k = max(lam_k, v)
    F = np.sum(np.where(bp <= lam_k, d * d, 0.0))
    Ahi = np.sum(np.where(bp > lam_k, a * a, 0.0))
    lam = np.sqrt(max(r * r - F, 0.0) / Ahi)
    return float(np.sum(a * np.minimum(lam * a, d)))


def _random_tr(rng, N, inf_frac=0.2, zero_frac=0.1, atbound_frac=0.1):
    a = np.abs(rng.standard_normal(N)) * 10 ** rng.uniform(-2, 2, N)
    a[rng.random(N) < zero_frac] = 0.0
    d = np.abs(rng.standard_normal(N)) * 10 ** rng.uniform(-2, 2, N)
    d[rng.random(N) < inf_frac] = np.inf
    d[rng.random(N) < atbound_frac] = 0.0
    return a, d


@pytest.mark.parametrize("seed", range(40))
def test_trust_region_matches_sort_and_scan(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(1, 300))
    a, d = _random_tr(rng, N, inf_frac=[0.0, 0.2, 0.9][seed % 3])
    fin = d[np.isfinite(d) & (a > 0)]
    full = np.sqrt(np.sum(fin ** 2)) if fin.size else 1.0
    for r in [1e-3 * full, 0.1 * full, 0.5 * full, 0.99 * full, 2 * full + 1]:
        val, lam = oracle.trust_region(a, d, r)
        ref = tr_sort_and_scan(a, d, r)
        assert val == pytest.approx(ref, rel=1e-12, abs=1e-300)


def test_trust_region_with_ties_and_duplicates():
    a = np.array([1.0, 1.0, 2.0, 2.0, 0.5, 0.5, 3.0])
    d = np.array([1.0, 1.0, 2.0, 2.0, 0.5, 0.5, 3.0])  # all breakpoints = 1
    for r in [0.1, 1.0, 2.5, 4.0, 4.5, 10.0]:
        val, _ = oracle.trust_region(a, d, r)
        assert val == pytest.approx(tr_sort_and_scan(a, d, r), rel=1e-13)


def test_trust_region_full_box_branch():
    """First line of Algorithm 2: when the bound lies inside the ball the
    answer is the bound itself (lambda = inf)."""
    a = np.array([1.0, 2.0, 3.0])
    d = np.array([0.1, 0.2, 0.3])
    val, lam = oracle.trust_region(a, d, 1.0)
    assert np.isinf(lam)
    assert val == pytest.approx(0.1 + 0.4 + 0.9)


def test_trust_region_no_bounds_is_norm():
    """With no finite bound the maximiser is r g/||g||: value = r ||g||."""
    rng = np.random.default_rng(5)
    a = np.abs(rng.standard_normal(50))
    d = np.full(50, np.inf)
    val, lam = oracle.trust_region(a, d, 0.7)
    assert val == pytest.approx(0.7 * np.linalg.norm(a), rel=1e-14)
    assert lam == pytest.approx(0.7 / np.linalg.norm(a), rel=1e-14)


def test_trust_region_zero_radius_and_zero_gradient():
    assert oracle.trust_region([1.0, 2.0], [1.0, np.inf], 0.0)[0] == 0.0
    assert oracle.trust_region([0.0, 0.0], [1.0, np.inf], 1.0)[0] == 0.0


@pytest.mark.parametrize("seed", range(12))
def test_trust_region_against_slsqp(seed):
    """Tiny problems solved by a general constrained optimiser in the
    original coordinates: min g'z~ s.t. lo <= z~ <= hi, ||z~ - z|| <= r."""
    rng = np.random.default_rng(100 + seed)
    N = 4
    z = rng.uniform(-1, 1, N)
    lo = z - rng.uniform(0, 1, N)
    hi = z + rng.uniform(0, 1, N)
    lo[rng.random(N) < 0.3] = -np.inf
    hi[rng.random(N) < 0.3] = np.inf
    g = rng.standard_normal(N)
    r = float(rng.uniform(0.2, 1.5))
    bnds = [(None if np.isinf(l_) else l_, None if np.isinf(h_) else h_)
            for l_, h_ in zip(lo, hi)]
    cons = [{"type": "ineq", "fun": lambda w: r * r - np.sum((w - z) ** 2)}]
    best = None
    for trial in range(6):
        w0 = z + 0.1 * r * rng.standard_normal(N)
        w0 = np.clip(w0, lo, hi)
        res = minimize(lambda w: g @ w, w0, bounds=bnds, constraints=cons,
                       method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
        w = res.x
        ok = (np.linalg.norm(w - z) <= r * (1 + 1e-7)
              and np.all(w >= lo - 1e-9) and np.all(w <= hi + 1e-9))
        if ok and (best is None or g @ w < best):
            best = g @ w
    assert best is not None
    ref = g @ z - best
    a = np.abs(g)
    d = np.where(g > 0, z - lo, np.where(g < 0, hi - z, 0.0))
    val, _ = oracle.trust_region(a, d, r)
    assert val == pytest.approx(ref, rel=1e-6, abs=1e-9)


# ------------------------------------------------------------------ gap ---

def _free_lp(seed, m=20, n=30):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) * (rng.random((m, n)) < 0.3)
    return lp_from_dense(A, rng.standard_normal(m), rng.standard_normal(n),
                         [-np.inf] * n, [np.inf] * n)


@pytest.mark.parametrize("seed", range(5))
def test_gap_unbounded_equals_operator_norm(seed):
    """Lemma example:bilinear, eq. bilinear-1: with Z the whole space,
    rho_r(z) = ||F(z)|| = ||(c - A'y, Ax - b)|| for every r > 0."""
    lp = _free_lp(seed)
    A = dense_A(lp)
    o = oracle.Oracle(lp, eta=0.1)
    rng = np.random.default_rng(seed + 50)
    x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    F = np.concatenate([lp.c - A.T @ y, A @ x - lp.b])
    for r in [1e-3, 0.5, 7.0]:
        rho, _ = o.gap_at(x, y, r)
        assert rho == pytest.approx(np.linalg.norm(F), rel=1e-13)


@pytest.mark.parametrize("case", range(6))
def test_gap_zero_at_planted_optimum(case):
    """Proposition prop:rho-duality-gap: rho_r(z*) = 0 at a saddle point."""
    lp = planted_cases()[case]
    o = oracle.Oracle(lp, eta=0.1)
    scale = 1 + np.abs(lp.c).max() + np.abs(lp.b).max()
    for r in [1e-2, 1.0, 100.0]:
        rho, _ = o.gap_at(lp.x_star, lp.y_star, r)
        assert abs(rho) <= 1e-12 * scale


@pytest.mark.parametrize("case", range(6))
def test_gap_monotone_in_radius(case):
    """Fact fact:monotone-r-rho-r and Proposition prop:basic-properties:
    r rho_r is non-decreasing and rho_r non-increasing in r."""
    lp = planted_cases()[case]
    o = oracle.Oracle(lp, eta=0.1)
    rng = np.random.default_rng(case)
    x = np.clip(lp.x_star + rng.standard_normal(lp.n), lp.l, lp.u)
    y = lp.y_star + rng.standard_normal(lp.m)
    y[lp.row_kind == 1] = np.abs(y[lp.row_kind == 1])
    rs = np.geomspace(1e-4, 1e3, 40)
    rho = np.array([o.gap_at(x, y, r)[0] for r in rs])
    assert np.all(np.diff(rho) <= 1e-12 * (1 + rho[:-1]))
    rr = rs * rho
    assert np.all(np.diff(rr) >= -1e-12 * (1 + rr[:-1]))


@pytest.mark.parametrize("seed", range(6))
def test_gap_lemma3_kkt_bound(seed):
    """Lemma lem:bound-kkt-error in standard form (x >= 0, Ax = b):
    ||(h - Kz)^+|| <= rho_r(z) sqrt(1 + R^2) for ||z|| <= R, r <= R."""
    rng = np.random.default_rng(300 + seed)
    m, n = 6, 10
    A = rng.standard_normal((m, n))
    xs = np.abs(rng.standard_normal(n)) * (rng.random(n) < 0.6)
    b = A @ xs
    c = A.T @ rng.standard_normal(m) + np.where(xs > 0, 0.0, rng.uniform(0.1, 1, n))
    lp = lp_from_dense(A, b, c, [0.0] * n, [np.inf] * n)
    o = oracle.Oracle(lp, eta=0.1, kkt_kind=oracle.KKT_PAPER_ABS)
    for _ in range(10):
        x = np.abs(rng.standard_normal(n))
        y = rng.standard_normal(m)
        R = np.sqrt(x @ x + y @ y) * (1 + rng.random())
        r = R * rng.uniform(0.05, 1.0)
        rho, _ = o.gap_at(x, y, r)
        kkt = o.kkt_at(x, y)[5]
        assert kkt <= rho * np.sqrt(1 + R * R) * (1 + 1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_gap_against_lagrangian_definition(seed):
    """eq. rhorz evaluated from its definition: maximise L(x, y~) - L(x~, y)
    with L = c'x - y'Ax + b'y over the ball intersected with Z, by a general
    optimiser, on tiny LPs with boxes, free variables and >= rows."""
    rng = np.random.default_rng(400 + seed)
    m, n = 2, 3
    A = rng.standard_normal((m, n))
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    l = np.array([0.0, -1.0, -np.inf])
    u = np.array([1.0, np.inf, np.inf])
    kind = np.array([0, 1], np.int8)
    lp = lp_from_dense(A, b, c, l, u, kind)
    o = oracle.Oracle(lp, eta=0.1)
    x = np.array([rng.uniform(0, 1), rng.uniform(-1, 2), rng.standard_normal()])
    y = np.array([rng.standard_normal(), abs(rng.standard_normal())])
    L = lambda xx, yy: c @ xx - yy @ (A @ xx) + b @ yy
    r = float(rng.uniform(0.3, 2.0))
    z = np.concatenate([x, y])
    bnds = [(0, 1), (-1, None), (None, None), (None, None), (0, None)]
    cons = [{"type": "ineq", "fun": lambda w: r * r - np.sum((w - z) ** 2)}]
    best = -np.inf
    for trial in range(8):
        w0 = z + 0.2 * r * rng.standard_normal(5)
        w0 = np.clip(w0, [0, -1, -np.inf, -np.inf, 0], [1, np.inf, np.inf, np.inf, np.inf])
        res = minimize(lambda w: -(L(x, w[3:]) - L(w[:3], y)), w0, bounds=bnds,
                       constraints=cons, method="SLSQP",
                       options={"ftol": 1e-14, "maxiter": 500})
        w = res.x
        feasible = (np.linalg.norm(w - z) <= r * (1 + 1e-7) and w[0] >= -1e-9
                    and w[0] <= 1 + 1e-9 and w[1] >= -1 - 1e-9 and w[4] >= -1e-9)
        if feasible:
            best = max(best, L(x, w[3:]) - L(w[:3], y))
    assert np.isfinite(best)
    rho, _ = o.gap_at(x, y, r)
    assert rho == pytest.approx(best / r, rel=1e-6, abs=1e-9)


def test_gap_primal_weight_is_rescaled_euclidean():
    """With primal weight omega the gap is the plain Euclidean gap of the
    rescaled space x^ = sqrt(omega) x, y^ = y / sqrt(omega) (footnote to
    eq. PDHG-update), in which the LP has data (c/sqrt(w), A/1, b*sqrt(w))
    up to the coupling: checked against the omega = 1 gap of that LP."""
    rng = np.random.default_rng(9)
    m, n = 8, 12
    A = rng.standard_normal((m, n)) * (rng.random((m, n)) < 0.5)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    l = np.where(rng.random(n) < 0.5, 0.0, -np.inf)
    u = np.where(rng.random(n) < 0.5, 2.0, np.inf)
    kind = (rng.random(m) < 0.5).astype(np.int8)
    w = 3.7
    sw = np.sqrt(w)
    lp = lp_from_dense(A, b, c, l, u, kind)
    # rescaled LP: x^ = sw x, y^ = y / sw; c'x = (c/sw)'x^, y'Ax = y^'Ax^,
    # b'y = (b sw)'y^
    lp2 = lp_from_dense(A, b * sw, c / sw, l * sw, u * sw, kind)
    o1 = oracle.Oracle(lp, eta=0.1, omega=w)
    o2 = oracle.Oracle(lp2, eta=0.1, omega=1.0)
    x = np.clip(rng.standard_normal(n), l, u)
    y = rng.standard_normal(m)
    y[kind == 1] = np.abs(y[kind == 1])
    for r in [0.1, 1.0, 10.0]:
        g1, _ = o1.gap_at(x, y, r)
        g2, _ = o2.gap_at(x * sw, y / sw, r)
        assert g1 == pytest.approx(g2, rel=1e-12)
