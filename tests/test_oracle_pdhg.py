"""Pins for the oracle's PDHG step, averaging and fixed-length restarts.

Each test compares the oracle with something it does not compute itself:
the paper's closed-form linear dynamics for bilinear problems, the exact
fixed point of a planted LP, and the non-expansiveness of PDHG.
"""
import numpy as np
import pytest

import oracle
from tests.lp_cases import bilinear_lp, dense_A, planted_cases


def _pdhg_matrix(eta, s):
    # eq. PDHG_simple for L(x,y) = s*x*y (scalar A = s)
    return np.array([[1.0, -eta * s], [eta * s, 1.0 - 2.0 * eta * eta * s * s]])


def test_figure1_bilinear_trajectory():
    """Fig. 1: L = xy, eta = 0.2; the first 50 PDHG iterates equal P^t z0."""
    lp = bilinear_lp([1.0])
    o = oracle.Oracle(lp, eta=0.2, mode=oracle.MODE_NONE)
    z0 = np.array([1.0, 0.5])
    o.set_point(z0[:1], z0[1:])
    P = _pdhg_matrix(0.2, 1.0)
    z = z0.copy()
    for t in range(1, 51):
        o.step(1)
        z = P @ z
        x, y = o.get(0)
        np.testing.assert_allclose([x[0], y[0]], z, rtol=0, atol=1e-14)
    # the running average over the 50 iterates
    zs = [np.linalg.matrix_power(P, t) @ z0 for t in range(1, 51)]
    xa, ya = o.get(1)
    np.testing.assert_allclose([xa[0], ya[0]], np.mean(zs, axis=0), atol=1e-14)


def test_figure1_fixed_restart_length_25():
    """Fig. 1's restarted run: fixed restart length 25 restarts to the
    average of the 25 iterates of the window (Algorithm 1)."""
    lp = bilinear_lp([1.0])
    o = oracle.Oracle(lp, eta=0.2, mode=oracle.MODE_FIXED, fixed_len=25)
    z0 = np.array([1.0, 0.5])
    o.set_point(z0[:1], z0[1:])
    P = _pdhg_matrix(0.2, 1.0)
    anchor = z0
    for window in range(2):
        zs = [np.linalg.matrix_power(P, t) @ anchor for t in range(1, 26)]
        for t in range(25):
            o.step(1)
            if t < 24:
                x, y = o.get(0)
                np.testing.assert_allclose([x[0], y[0]], zs[t], atol=1e-14)
        anchor = np.mean(zs, axis=0)
        x, y = o.get(0)
        np.testing.assert_allclose([x[0], y[0]], anchor, atol=1e-14)
        x0, y0 = o.get(2)
        np.testing.assert_allclose([x0[0], y0[0]], anchor, atol=1e-14)
        assert o.info()["restarts"] == window + 1
        assert o.info()["t"] == 0
    # restarted average is much closer to the optimum (0, 0) than the plain run
    plain = np.linalg.matrix_power(P, 50) @ z0
    assert np.linalg.norm(anchor) < 0.5 * np.linalg.norm(plain)


def test_bilinear_decay_rate_in_eigenbasis():
    """eq. lin-converge / eq. lambda-i-abs: in the basis Q_i the squared
    norm of each 2-d block decays by exactly (1 - eta^2 s_i^2) per step."""
    s = np.array([0.3, 0.7, 1.1, 1.9, 2.5])
    eta = 0.9 / s.max()
    lp = bilinear_lp(s)
    o = oracle.Oracle(lp, eta=eta, mode=oracle.MODE_NONE)
    rng = np.random.default_rng(0)
    x0, y0 = rng.standard_normal(5), rng.standard_normal(5)
    o.set_point(x0, y0)

    def qinv_norm2(x, y):
        out = []
        for i, si in enumerate(s):
            w = np.sqrt(1 - eta * eta * si * si)
            Q = np.array([[eta * si - 1j * w, eta * si + 1j * w], [1, 1]])
            zt = np.linalg.solve(Q, np.array([x[i], y[i]], dtype=complex))
            out.append(np.vdot(zt, zt).real)
        return np.array(out)

    base = qinv_norm2(x0, y0)
    for t in range(1, 41):
        o.step(1)
        x, y = o.get(0)
        np.testing.assert_allclose(qinv_norm2(x, y),
                                   base * (1 - eta * eta * s * s) ** t,
                                   rtol=1e-11)


@pytest.mark.parametrize("case", range(6))
def test_planted_optimum_is_fixed_point(case):
    """A planted KKT point is a fixed point of one PDHG step."""
    lp = planted_cases()[case]
    o = oracle.Oracle(lp, mode=oracle.MODE_NONE)
    xo, yo = o.pdhg_map(lp.x_star, lp.y_star)
    np.testing.assert_allclose(xo, lp.x_star, atol=1e-12)
    np.testing.assert_allclose(yo, lp.y_star, atol=1e-12)


def _mnorm2(dx, dy, A, tau, sigma):
    # PDHG norm of Proposition prop:assumption-one-holds for the LP coupling
    # -y'Ax, written with separate primal and dual steps
    return dx @ dx / tau + 2.0 * dy @ (A @ dx) + dy @ dy / sigma


@pytest.mark.parametrize("case", range(6))
def test_nonexpansive_in_pdhg_norm(case):
    """Proposition prop:convergence (i): ||z^{t+1} - z*|| <= ||z^t - z*|| in
    the PDHG norm, for the planted z*, along 300 iterations."""
    lp = planted_cases()[case]
    A = dense_A(lp)
    o = oracle.Oracle(lp, mode=oracle.MODE_NONE, omega=[1.0, 1.0, 4.0, 0.25, 1.0, 2.0][case])
    inf = o.info()
    prev = None
    for _ in range(300):
        x, y = o.get(0)
        d = _mnorm2(x - lp.x_star, y - lp.y_star, A, inf["tau"], inf["sigma"])
        assert d >= -1e-12
        if prev is not None:
            assert d <= prev * (1 + 1e-12) + 1e-13
        prev = d
        o.step(1)


def test_average_is_mean_of_window():
    """Algorithm 1, average line: z-bar is the mean of the window's iterates."""
    lp = planted_cases()[2]
    o = oracle.Oracle(lp, mode=oracle.MODE_NONE)
    xs, ys = [], []
    for _ in range(17):
        o.step(1)
        x, y = o.get(0)
        xs.append(x)
        ys.append(y)
    xa, ya = o.get(1)
    np.testing.assert_allclose(xa, np.mean(xs, axis=0), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(ya, np.mean(ys, axis=0), rtol=1e-14, atol=1e-15)


def test_initial_point_is_projected_origin():
    lp = planted_cases()[3]
    o = oracle.Oracle(lp)
    x, y = o.get(0)
    np.testing.assert_array_equal(x, np.clip(0.0, lp.l, lp.u))
    np.testing.assert_array_equal(y, 0.0)


def test_iterates_stay_feasible():
    lp = planted_cases()[4]
    o = oracle.Oracle(lp, mode=oracle.MODE_ADAPTIVE)
    for _ in range(10):
        o.solve(30, 0.0)
        x, y = o.get(0)
        assert np.all(x >= lp.l) and np.all(x <= lp.u)
        assert np.all(y[lp.row_kind == 1] >= 0)
