"""Pins for the primal weight in the oracle (Section 7: primal step
eta/omega, dual step eta*omega) and for its weight search.

The weight is pinned by an exact change of variables: PDHG with weight
omega on (c, A, b) is PDHG with weight 1 on (c/omega, A, b) with the dual
iterate scaled, y = omega * y~.  (The x update reads
x - (eta/omega)(c - A'y) = x - eta(c/omega - A'y~); the y update divided by
omega is y~ + eta(b - A(2x+ - x)), and the projection onto the dual cone
commutes with positive scaling.)  With omega a power of two every rounding
step agrees, so the two runs match bit for bit; swapping the two step sizes
or scaling the wrong vector breaks it.
"""
import numpy as np
import pytest

import oracle
from paper_2105_12715_amd import lpgen
from tests.lp_cases import planted_cases


def _scaled_c(lp, f):
    return lpgen.LP(**{**lp.__dict__, "c": np.asarray(lp.c) * f})


@pytest.mark.parametrize("omega", [4.0, 0.0625, 1024.0])
@pytest.mark.parametrize("case", [0, 2, 4])
def test_weight_is_a_change_of_variables(case, omega):
    lp = planted_cases()[case]
    eta = 0.5 * oracle.Oracle(lp).info()["eta"]
    a = oracle.Oracle(lp, eta=eta, omega=omega, mode=oracle.MODE_NONE)
    b = oracle.Oracle(_scaled_c(lp, 1.0 / omega), eta=eta, omega=1.0, mode=oracle.MODE_NONE)
    for _ in range(4):
        a.step(50)
        b.step(50)
        xa, ya = a.get(0)
        xb, yb = b.get(0)
        np.testing.assert_array_equal(xa, xb)
        np.testing.assert_array_equal(ya, omega * yb)
    # the running sums follow the same change of variables
    xa, ya = a.get(1)
    xb, yb = b.get(1)
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(ya, omega * yb)


def test_weight_changes_the_iterates():
    """Guards the pin above against a weight that is ignored."""
    lp = planted_cases()[0]
    eta = oracle.Oracle(lp).info()["eta"]
    a = oracle.Oracle(lp, eta=eta, omega=1.0, mode=oracle.MODE_NONE)
    b = oracle.Oracle(lp, eta=eta, omega=4.0, mode=oracle.MODE_NONE)
    a.step(20)
    b.step(20)
    assert np.linalg.norm(a.get(0)[0] - b.get(0)[0]) > 1e-6


def test_search_without_iterations_ties_to_the_first_weight():
    """At iteration 0 every copy sits at the same initial point, so every
    criterion value is the same and the first weight wins."""
    lp = planted_cases()[1]
    om = [4.0 ** k for k in range(-5, 6)]
    parts, best, xs, ys = oracle.weight_search(lp, om, 0, 0.1)
    assert best == 0
    assert np.all(parts[:, 5] == parts[0, 5])
    assert np.all(xs == xs[0]) and np.all(ys == 0.0)


def test_search_criterion_is_the_paper_kkt_of_the_last_iterate():
    """Each row of the search is the KKT error of the last iterate of an
    independent run, and the pick is the smallest ||(h - Kz)^+||_2."""
    lp = planted_cases()[2]
    eta = oracle.Oracle(lp).info()["eta"]
    om = [0.25, 1.0, 4.0]
    parts, best, xs, ys = oracle.weight_search(lp, om, 200, eta)
    for w, o in enumerate(om):
        r = oracle.Oracle(lp, eta=eta, omega=o, mode=oracle.MODE_NONE)
        r.step(200)
        np.testing.assert_array_equal(parts[w], r.kkt(0))
        np.testing.assert_array_equal(xs[w], r.get(0)[0])
    assert best == int(np.argmin(parts[:, 5]))
    # the criterion is zero at a planted optimum, so it is a distance to it
    o = oracle.Oracle(lp, eta=eta)
    assert o.kkt_at(lp.x_star, lp.y_star)[5] <= 1e-9 * (1 + np.abs(lp.c).sum())
