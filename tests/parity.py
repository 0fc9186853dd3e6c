"""Comparison helpers of the GPU parity tests.

A GPU point matches the oracle's at tolerance `tol` when both hold:
  - the norm bound  ||z_gpu - z_cpu||_2 <= tol ||z_cpu||_2, and
  - the coordinate bound  |z_gpu,i - z_cpu,i| <= tol (|z_cpu,i| + ||z_cpu||_inf)
    for every i.
The second one catches a single coordinate that is far off on an iterate
with millions of coordinates, which the norm bound alone would let through.
The ||z||_inf term keeps the bound meaningful for coordinates at or near
zero, where sums taken in another order differ by an absolute rounding
error of the size of the vector's largest terms.
"""
from __future__ import annotations

import numpy as np


def deviation(got, ref):
    """(norm-relative deviation, worst coordinate ratio, its index)."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    assert got.shape == ref.shape, (got.shape, ref.shape)
    if ref.size == 0:
        return 0.0, 0.0, -1
    diff = np.abs(got - ref)
    nref = np.linalg.norm(ref)
    norm_rel = float(np.linalg.norm(got - ref) / (nref if nref > 0 else 1.0))
    inf = float(np.max(np.abs(ref)))
    scale = np.abs(ref) + (inf if inf > 0 else 1.0)
    ratio = diff / scale
    # NaN anywhere is a mismatch
    ratio = np.where(np.isnan(ratio), np.inf, ratio)
    i = int(np.argmax(ratio))
    return norm_rel, float(ratio[i]), i


def assert_points_match(got, ref, tol, what=""):
    """Norm and per-coordinate bounds (module docstring); on failure the
    message names the worst coordinate and both values."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    norm_rel, worst, i = deviation(got, ref)
    ok = norm_rel <= tol and worst <= tol
    assert ok, (f"{what}: norm-relative deviation {norm_rel:.3e}, worst coordinate {i} "
                f"(gpu {got[i]!r}, oracle {ref[i]!r}) at {worst:.3e} of its bound, "
                f"tolerance {tol:g}")
    return norm_rel, worst


def assert_within_sum_bound(got, ref, absA, v, what=""):
    """Row sums of a sparse product taken in two summation orders agree
    within the bound that holds for any order: |a - b| <= 2 k u sum_j
    |a_ij v_j| for a row of k entries (u = 2^-53).  absA: scipy CSR of |A|
    (or |A'|)."""
    k = np.diff(absA.indptr).astype(float)
    mag = absA @ np.abs(np.asarray(v, dtype=np.float64))
    bound = 2.0 * k * 2.0 ** -53 * mag
    err = np.abs(np.asarray(got, dtype=np.float64) - np.asarray(ref, dtype=np.float64))
    bad = np.flatnonzero(~(err <= bound))
    assert bad.size == 0, (f"{what}: {bad.size} rows outside the summation bound; first "
                           f"row {bad[0]}: |diff| {err[bad[0]]:.3e} > {bound[bad[0]]:.3e}")
