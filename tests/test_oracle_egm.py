"""Pins for the oracle's extragradient method (eq. extra-gradient-update)
inside Algorithm 1.

For the bilinear saddle L(x, y) = s x y (no constraints) the operator is
F(z) = (s y, -s x), so one step is linear: with a = eta s the target is
N z = (x - a y, y + a x) and the new iterate M z = ((1-a^2) x - a y,
a x + (1-a^2) y).  M is a scaled rotation with |M z| = sqrt(1 - a^2 + a^4)
|z|: the last iterate contracts, unlike PDHG's.  A planted optimum is a
fixed point of the step, and restarted runs reach the planted objective.
"""
import numpy as np
import pytest

import oracle
from tests.lp_cases import bilinear_lp, planted_cases


def _egm(lp, **kw):
    return oracle.Oracle(lp, method=oracle.METHOD_EGM, **kw)


@pytest.mark.parametrize("s,eta", [(1.0, 0.2), (0.5, 0.9), (2.0, 0.3)])
def test_bilinear_closed_form(s, eta):
    lp = bilinear_lp([s])
    o = _egm(lp, eta=eta, mode=oracle.MODE_NONE)
    z0 = np.array([1.0, 0.5])
    o.set_point(z0[:1], z0[1:])
    a = eta * s
    M = np.array([[1 - a * a, -a], [a, 1 - a * a]])
    N = np.array([[1.0, -a], [a, 1.0]])
    z = z0.copy()
    targets = []
    for t in range(1, 41):
        targets.append(N @ z)
        o.step(1)
        z = M @ z
        x, y = o.get(0)
        np.testing.assert_allclose([x[0], y[0]], z, rtol=0, atol=1e-14)
    xa, ya = o.get(1)
    np.testing.assert_allclose([xa[0], ya[0]], np.mean(targets, axis=0), atol=1e-14)


def test_bilinear_last_iterate_contracts():
    """|z^t| = (1 - a^2 + a^4)^(t/2) |z^0| for every coordinate pair."""
    s = np.array([1.0, 0.25, 3.0])
    eta = 0.3
    lp = bilinear_lp(s)
    o = _egm(lp, eta=eta, mode=oracle.MODE_NONE)
    x0 = np.array([1.0, -2.0, 0.5])
    y0 = np.array([0.3, 1.0, -1.0])
    o.set_point(x0, y0)
    T = 25
    o.step(T)
    x, y = o.get(0)
    a = eta * s
    rate = (1 - a * a + a ** 4) ** (T / 2)
    np.testing.assert_allclose(np.hypot(x, y), rate * np.hypot(x0, y0), rtol=1e-12)


@pytest.mark.parametrize("case", range(6))
def test_planted_optimum_is_a_fixed_point(case):
    lp = planted_cases()[case]
    o = _egm(lp, mode=oracle.MODE_NONE)
    o.set_point(lp.x_star, lp.y_star)
    o.step(1)
    x, y = o.get(0)
    scale = 1 + np.abs(lp.x_star).max() + np.abs(lp.y_star).max()
    assert np.abs(x - lp.x_star).max() <= 1e-12 * scale
    assert np.abs(y - lp.y_star).max() <= 1e-12 * scale
    # the target of that step is the optimum too (it is the window's average)
    xa, ya = o.get(1)
    assert np.abs(xa - lp.x_star).max() <= 1e-12 * scale


def test_a_point_off_the_optimum_moves():
    lp = planted_cases()[2]
    o = _egm(lp, mode=oracle.MODE_NONE)
    o.step(1)
    assert np.abs(o.get(0)[0] - o.get(2)[0]).max() > 1e-6


@pytest.mark.parametrize("case", [0, 2, 4])
@pytest.mark.parametrize("mode", [oracle.MODE_ADAPTIVE, oracle.MODE_FLEXIBLE])
def test_restarted_egm_reaches_the_planted_objective(case, mode):
    lp = planted_cases()[case]
    o = _egm(lp, mode=mode)
    res = o.solve(400_000, 1e-8)
    assert res["status"] == 0
    obj = lp.objective_star()
    assert abs(res["pobj"] - obj) <= 1e-6 * (1 + abs(obj))
    assert res["restarts"] >= 1
