"""Pins for the oracle's reverse pass through K unrolled restarted-PDHG
iterations (gradient of |x_K - x_target|^2 with respect to c, b and the
values of A): central finite differences on coordinates whose perturbed
runs take the same branch (masks and restarts), the dot-product identity
against the oracle's tangent pass, and exactness on a bilinear problem,
where the K-step map is linear."""
import numpy as np
import pytest

import oracle
from paper_2105_12715_amd import lpgen
from tests.lp_cases import bilinear_lp


def _perturbed(lp, kind, idx, h):
    c, b, v = lp.c.copy(), lp.b.copy(), lp.vals.copy()
    if kind == "c":
        c[idx] += h
    elif kind == "b":
        b[idx] += h
    else:
        v[idx] += h
    return lpgen.LP(**{**lp.__dict__, "c": c, "b": b, "vals": v})


def _loss(lp, eta, mode, K, xt):
    o = oracle.Oracle(lp, eta=eta, mode=mode)
    xk = o.unrolled_value(K)
    return float(np.sum((xk - xt) ** 2)), o.branch_signature(K)


@pytest.mark.parametrize("mode", [oracle.MODE_ADAPTIVE, oracle.MODE_FLEXIBLE, oracle.MODE_NONE])
def test_gradient_matches_central_differences(mode):
    lp = lpgen.bernoulli_lp(31, 12, 24, 0.3, lpgen.BOX01, ge_frac=0.3)
    K = 150
    eta = oracle.Oracle(lp).info()["eta"]
    xt = np.random.default_rng(5).uniform(0, 1, lp.n)
    o = oracle.Oracle(lp, eta=eta, mode=mode)
    loss, gc, gb, gA, xk = o.unrolled_grad(K, xt)
    base_sig = o.branch_signature(K)
    assert loss == pytest.approx(np.sum((xk - xt) ** 2))
    rng = np.random.default_rng(7)
    h = 1e-6
    checked = 0
    for kind, size, g in (("c", lp.n, gc), ("b", lp.m, gb), ("A", lp.nnz, gA)):
        for idx in rng.choice(size, size=min(8, size), replace=False):
            lp_p, lp_m = _perturbed(lp, kind, idx, h), _perturbed(lp, kind, idx, -h)
            fp, sp = _loss(lp_p, eta, mode, K, xt)
            fm, sm = _loss(lp_m, eta, mode, K, xt)
            if sp != base_sig or sm != base_sig:
                continue  # a mask or restart flips between the runs
            fd = (fp - fm) / (2 * h)
            assert g[idx] == pytest.approx(fd, rel=1e-5, abs=1e-7), (kind, idx)
            checked += 1
    assert checked >= 12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dot_product_identity_with_tangent_pass(seed):
    """<J v, w> = <v, J' w> with w = 2 (x_K - x_target)."""
    lp = [lpgen.small_dense(1),
          lpgen.column_count_lp(13, 60, 120, per_col=5, bounds="mixed_inf", ge_frac=0.5),
          lpgen.bernoulli_lp(11, 30, 60, 0.15, lpgen.BOX01, ge_frac=0.4)][seed]
    K = 400
    mode = [oracle.MODE_ADAPTIVE, oracle.MODE_FLEXIBLE, oracle.MODE_FIXED][seed]
    eta = oracle.Oracle(lp).info()["eta"]
    rng = np.random.default_rng(seed)
    xt = rng.uniform(0, 1, lp.n)
    o = oracle.Oracle(lp, eta=eta, mode=mode, fixed_len=64)
    loss, gc, gb, gA, xk = o.unrolled_grad(K, xt)
    dc, db, dA = rng.standard_normal(lp.n), rng.standard_normal(lp.m), rng.standard_normal(lp.nnz)
    jv = o.unrolled_tangent(K, dc, db, dA)
    lhs = jv @ (2 * (xk - xt))
    rhs = dc @ gc + db @ gb + dA @ gA
    assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-12)


def test_bilinear_map_is_linear_so_gradient_is_exact():
    """Without bounds and restarts the K-step map is linear in (c, b): a
    finite difference with h = 1 is exact up to rounding."""
    lp = bilinear_lp([0.4, 0.9, 1.3])
    lp = lpgen.LP(**{**lp.__dict__, "c": np.array([0.3, -0.2, 0.5]),
                     "b": np.array([0.1, 0.7, -0.4])})
    K, eta = 60, 0.5
    xt = np.array([0.2, -0.1, 0.3])
    o = oracle.Oracle(lp, eta=eta, mode=oracle.MODE_NONE)
    loss, gc, gb, gA, xk = o.unrolled_grad(K, xt)
    for kind, size, g in (("c", 3, gc), ("b", 3, gb)):
        for idx in range(size):
            fp, _ = _loss(_perturbed(lp, kind, idx, 1.0), eta, oracle.MODE_NONE, K, xt)
            fm, _ = _loss(_perturbed(lp, kind, idx, -1.0), eta, oracle.MODE_NONE, K, xt)
            assert g[idx] == pytest.approx((fp - fm) / 2.0, rel=1e-10, abs=1e-13)
