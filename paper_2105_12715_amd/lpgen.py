"""Seeded synthetic LP workloads with a planted optimum.

This module only draws inputs. It holds none of the solver's arithmetic and
is the one piece shared by the HIP path, the CPU oracle and the tests.

Construction (the planted-optimum recipe): pick a sparsity pattern and values
for ``A``, a bound class per variable, a status per variable (at lower bound,
at upper bound or interior), a primal point ``x*`` consistent with the
status, a dual point ``y*`` and reduced costs ``r`` that are positive at lower
bounds, negative at upper bounds and zero elsewhere.  Then ``c = A^T y* + r``
and ``b = A x*`` make ``(x*, y*)`` satisfy the KKT conditions of

    min c^T x  s.t.  A x = b (rows of kind 0),  A x >= b (rows of kind 1),
                     l <= x <= u.

Draw order is fixed: pattern, values, bound classes, status, x*, y*, r.
All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.sparse as sp

INF = np.inf

# bound classes: (l, u)
BOX01 = (0.0, 1.0)
BOX010 = (0.0, 10.0)
LOWER0 = (0.0, INF)
UPPER0 = (-INF, 0.0)
FREE = (-INF, INF)
BOXM11 = (-1.0, 1.0)


@dataclasses.dataclass
class LP:
    """One LP in CSR form plus its planted solution."""
    m: int
    n: int
    row_ptr: np.ndarray   # int32, m+1
    col_idx: np.ndarray   # int32, nnz
    vals: np.ndarray      # float64, nnz
    c: np.ndarray         # float64, n
    b: np.ndarray         # float64, m
    l: np.ndarray         # float64, n (may hold -inf)
    u: np.ndarray         # float64, n (may hold +inf)
    row_kind: np.ndarray  # int8, m (0: equality, 1: >=)
    x_star: np.ndarray
    y_star: np.ndarray
    r_star: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy_csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals, self.col_idx, self.row_ptr),
                             shape=(self.m, self.n))

    def objective_star(self) -> float:
        return float(np.dot(self.c, self.x_star))


def _distinct_rows_per_column(rng, m: int, counts: np.ndarray):
    """For column j draw counts[j] distinct rows uniformly from [0, m)."""
    counts = np.minimum(counts.astype(np.int64), m)
    cols = np.repeat(np.arange(counts.size, dtype=np.int64), counts)
    rows = rng.integers(0, m, size=cols.size, dtype=np.int64)
    while True:
        key = cols * m + rows
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(ks.size, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        bad = order[dup]
        rows[bad] = rng.integers(0, m, size=bad.size, dtype=np.int64)
    return rows, cols


def _csr_from_coo(m, n, rows, cols, vals):
    a = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    a.sort_indices()
    return (a.indptr.astype(np.int32), a.indices.astype(np.int32),
            a.data.astype(np.float64))


def planted_lp(rng, m: int, n: int, rows, cols, vals, bound_l, bound_u,
               ge_frac: float = 0.0, p_lower: float = 0.3,
               p_upper: float = 0.2, name: str = "") -> LP:
    """Finish a planted LP once the pattern, values and bounds are drawn.

    ``rows``/``cols``/``vals`` describe A in coordinate form (distinct pairs).
    """
    row_ptr, col_idx, a_vals = _csr_from_coo(m, n, rows, cols, vals)
    l = np.asarray(bound_l, dtype=np.float64).copy()
    u = np.asarray(bound_u, dtype=np.float64).copy()
    # status: 0 lower, 1 upper, 2 interior
    s = rng.random(n)
    status = np.where(s < p_lower, 0, np.where(s < p_lower + p_upper, 1, 2))
    lfin, ufin = np.isfinite(l), np.isfinite(u)
    # a status that names a missing bound falls back to the other bound, else interior
    status = np.where((status == 1) & ~ufin, np.where(lfin, 0, 2), status)
    status = np.where((status == 0) & ~lfin, np.where(ufin, 1, 2), status)
    v = rng.uniform(0.1, 0.9, size=n)
    with np.errstate(invalid="ignore"):
        width = np.where(lfin & ufin, u - l, INF)
        interior = np.where(
            lfin & (width >= 1.0), l + v,
            np.where(lfin & ufin, l + v * width,
                     np.where(ufin, u - v, v - 0.5)))
    x_star = np.where(status == 0, l, np.where(status == 1, u, interior))
    y_star = rng.standard_normal(m)
    rmag = rng.uniform(0.1, 1.0, size=n)
    r_star = np.where(status == 0, rmag, np.where(status == 1, -rmag, 0.0))
    # inequality rows: a fraction of rows become A x >= b with y* >= 0;
    # half of them are slack (y* = 0, b below A x*)
    kind = np.zeros(m, dtype=np.int8)
    slack = np.zeros(m)
    if ge_frac > 0:
        g = rng.random(m) < ge_frac
        kind[g] = 1
        y_star = np.where(g, np.abs(y_star), y_star)
        sl = g & (rng.random(m) < 0.5)
        y_star = np.where(sl, 0.0, y_star)
        slack = np.where(sl, rng.uniform(0.1, 1.0, size=m), 0.0)
    A = sp.csr_matrix((a_vals, col_idx, row_ptr), shape=(m, n))
    c = A.T @ y_star + r_star
    b = A @ x_star - slack
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, vals=a_vals,
              c=np.ascontiguousarray(c, dtype=np.float64),
              b=np.ascontiguousarray(b, dtype=np.float64), l=l, u=u,
              row_kind=kind, x_star=x_star, y_star=y_star, r_star=r_star,
              name=name)


def bernoulli_lp(seed: int, m: int = 50, n: int = 100, density: float = 0.1,
                 bounds=BOX01, ge_frac: float = 0.0, name: str = "") -> LP:
    """Dense Bernoulli(density) pattern with N(0,1) values (the 50 x 100 case)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    rows, cols = np.nonzero(mask)
    vals = rng.standard_normal(rows.size)
    l = np.full(n, bounds[0])
    u = np.full(n, bounds[1])
    return planted_lp(rng, m, n, rows, cols, vals, l, u, ge_frac=ge_frac,
                      name=name or f"bernoulli{m}x{n}-s{seed}")


def column_count_lp(seed: int, m: int, n: int, counts=None, per_col: int = 0,
                    values: str = "normal", bounds: str = "box01",
                    ge_frac: float = 0.0, name: str = "") -> LP:
    """Each column gets a fixed or drawn number of distinct uniform rows.

    ``counts`` may be "powerlaw2" (P(k) proportional to k^-2 on 1..1000) or
    an array of n column counts.
    ``values``: "normal" (N(0,1)) or "loguniform" (random sign, 10^U(-3,3)).
    ``bounds``: "box01" (all [0,1]), "mix" (half [0,inf), half [0,10]) or
    "mixed_inf" (a mix of every bound class, for edge-case tests).
    """
    rng = np.random.default_rng(seed)
    if isinstance(counts, np.ndarray):
        cnt = counts.astype(np.int64)
    elif counts == "powerlaw2":
        k = np.arange(1, 1001, dtype=np.float64)
        p = k ** -2.0
        p /= p.sum()
        cnt = rng.choice(1000, size=n, p=p) + 1
    else:
        cnt = np.full(n, per_col, dtype=np.int64)
    rows, cols = _distinct_rows_per_column(rng, m, cnt)
    if values == "normal":
        vals = rng.standard_normal(rows.size)
    elif values == "loguniform":
        mag = 10.0 ** rng.uniform(-3.0, 3.0, size=rows.size)
        sgn = np.where(rng.random(rows.size) < 0.5, -1.0, 1.0)
        vals = sgn * mag
    else:
        raise ValueError(values)
    if bounds == "box01":
        l, u = np.zeros(n), np.ones(n)
    elif bounds == "mix":
        half = rng.permutation(n) < n // 2
        l = np.zeros(n)
        u = np.where(half, INF, 10.0)
    elif bounds == "mixed_inf":
        classes = [BOX01, LOWER0, UPPER0, FREE, BOXM11, BOX010]
        pick = rng.integers(0, len(classes), size=n)
        l = np.array([classes[i][0] for i in pick])
        u = np.array([classes[i][1] for i in pick])
    else:
        raise ValueError(bounds)
    return planted_lp(rng, m, n, rows, cols, vals, l, u, ge_frac=ge_frac,
                      name=name or f"cols{m}x{n}-s{seed}")


# ---------------------------------------------------------------------------
# The five workload shapes.
# ---------------------------------------------------------------------------

def small_dense(seed: int = 1) -> LP:
    """50 equality rows, 100 variables in [0,1], Bernoulli(0.1) N(0,1) entries."""
    return bernoulli_lp(seed, 50, 100, 0.1, BOX01, name=f"small50x100-s{seed}")


def medium(seed: int = 2) -> LP:
    """20,000 x 50,000, 10 distinct uniform rows per column, N(0,1) entries,
    half of the variables in [0,inf) and half in [0,10]."""
    return column_count_lp(seed, 20_000, 50_000, per_col=10, values="normal",
                           bounds="mix", name=f"medium20kx50k-s{seed}")


def large_powerlaw(seed: int = 3, m: int = 1_000_000, n: int = 2_000_000) -> LP:
    """1M x 2M with power-law column counts (exponent 2, 1..1000), random-sign
    log-uniform magnitudes in [1e-3, 1e3]; bounds as in the medium case."""
    return column_count_lp(seed, m, n, counts="powerlaw2", values="loguniform",
                           bounds="mix", name=f"large{m}x{n}-s{seed}")


def batch_member(i: int, base_seed: int = 4000) -> LP:
    """LP i of the uneven batch: m ~ U{200..20000}, n = 2m, 5 per column, [0,1]."""
    rng = np.random.default_rng(base_seed + i)
    m = int(rng.integers(200, 20_001))
    return column_count_lp(base_seed + i + 100_000, m, 2 * m, per_col=5,
                           values="normal", bounds="box01",
                           name=f"batch{i}-{m}x{2 * m}")


def diff_member(i: int, base_seed: int = 5000, m: int = 5000,
                n: int = 10_000) -> LP:
    """LP i of the differentiation batch: 5000 x 10000, 5 per column, [0,1]."""
    return column_count_lp(base_seed + i, m, n, per_col=5, values="normal",
                           bounds="box01", name=f"diff{i}-{m}x{n}")


def x_target(i: int, n: int, base_seed: int = 5100) -> np.ndarray:
    return np.random.default_rng(base_seed + i).uniform(0.0, 1.0, size=n)


# Sizes (rows, columns, entries) of the four LPs of Table 2.
TABLE2 = {
    "qap10": (1820, 4150, 18200),
    "qap15": (6330, 22275, 94950),
    "nug08-3rd": (19728, 20448, 139008),
    "nug20": (15240, 72600, 304800),
}


def paper_shaped(name: str, seed: int = 6000) -> LP:
    """Planted LP with exactly the size of a Table 2 instance: every column
    gets floor or ceil of nnz/n distinct uniform rows (the extra entries go
    to a random set of columns), values +1 or -1 with equal odds, x >= 0,
    all rows equalities.  A stand-in of the same shape, not the instance."""
    m, n, nnz = TABLE2[name]
    rng = np.random.default_rng(seed + sorted(TABLE2).index(name))
    base, extra = divmod(nnz, n)
    cnt = np.full(n, base, dtype=np.int64)
    cnt[rng.permutation(n)[:extra]] += 1
    rows, cols = _distinct_rows_per_column(rng, m, cnt)
    vals = np.where(rng.random(rows.size) < 0.5, -1.0, 1.0)
    l = np.zeros(n)
    u = np.full(n, INF)
    return planted_lp(rng, m, n, rows, cols, vals, l, u, name=f"{name}-shaped")
