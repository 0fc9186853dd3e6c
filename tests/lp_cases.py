"""Small LP builders shared by the tests (inputs only, no solver arithmetic)."""
import numpy as np

from paper_2105_12715_amd import lpgen


def lp_from_dense(A, b, c, l, u, kind=None, name="dense"):
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    rows, cols = np.nonzero(A)
    rp = np.zeros(m + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    order = np.lexsort((cols, rows))
    ci = cols[order].astype(np.int32)
    v = A[rows[order], cols[order]]
    kind = np.zeros(m, np.int8) if kind is None else np.asarray(kind, np.int8)
    f = lambda a: np.asarray([float(t) for t in a], dtype=np.float64)
    return lpgen.LP(m=m, n=n, row_ptr=rp, col_idx=ci, vals=v, c=f(c), b=f(b),
                    l=f(l), u=f(u), row_kind=kind, x_star=np.zeros(n),
                    y_star=np.zeros(m), r_star=np.zeros(n), name=name)


def bilinear_lp(diag):
    """L(x,y) = sum_i s_i x_i y_i written as the LP saddle c'x - y'Ax + b'y
    with A = -diag(s), c = b = 0 and no bounds."""
    s = np.asarray(diag, dtype=np.float64)
    k = s.size
    A = -np.diag(s)
    return lp_from_dense(A, np.zeros(k), np.zeros(k), [-np.inf] * k,
                         [np.inf] * k, name="bilinear")


def dense_A(lp):
    return lp.scipy_csr().toarray()


def planted_cases():
    """A spread of planted LPs: equality/>= rows and every bound class."""
    return [
        lpgen.small_dense(1),
        lpgen.small_dense(7),
        lpgen.bernoulli_lp(11, 30, 60, 0.15, lpgen.BOX01, ge_frac=0.4),
        lpgen.column_count_lp(12, 40, 90, per_col=4, bounds="mixed_inf"),
        lpgen.column_count_lp(13, 60, 120, per_col=5, bounds="mixed_inf",
                              ge_frac=0.5),
        lpgen.column_count_lp(14, 80, 200, per_col=6, bounds="mix"),
    ]
