"""ctypes binding of the plain FP64 CPU oracle (``pdhg_oracle.c``).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The HIP library
never calls into it and it never calls the HIP library.

Parity status of each oracle function (what pins it) is listed in the test
files under ``tests/test_oracle_*.py``; every function is pinned.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdhg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source with its per-coordinate loops and products on every host
# core (-DORC_OPENMP); bitwise equal results, used for the all-cores CPU
# baseline
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

MODE_NONE, MODE_ADAPTIVE, MODE_FLEXIBLE, MODE_FIXED = 0, 1, 2, 3
METHOD_PDHG, METHOD_EGM = 0, 1
KKT_RELATIVE, KKT_PAPER_ABS, KKT_MAX_ABS = 0, 1, 2
REC = 14

_lib = None
_lib_omp = None

_CFLAGS = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
           "-shared", "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused multiply-add, no fast math):
    the plain sequential build and the OpenMP build of the same source."""
    for lib, extra in ((_LIB, []), (_LIB_OMP, ["-DORC_OPENMP", "-fopenmp"])):
        if force or not os.path.exists(lib):
            tmp = lib + ".tmp"
            subprocess.check_call([*_CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, lib)
    return _LIB


def threads(parallel=True):
    """Threads the chosen build runs its parallel loops on (1: plain)."""
    return int(_load(parallel).orc_threads())


def _load(parallel=False):
    global _lib, _lib_omp
    if parallel:
        if _lib_omp is None:
            if not os.path.exists(_LIB_OMP):
                build(force=False)
            _lib_omp = _declare(C.CDLL(_LIB_OMP))
        return _lib_omp
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    _lib = _declare(C.CDLL(_LIB))
    return _lib


def _declare(L):
    P = C.c_void_p
    i64, i32, d = C.c_int64, C.c_int32, C.c_double
    L.orc_create.restype = P
    L.orc_create.argtypes = [i64, i64, P, P, P, P, P, P, P, P, d, d, d, i32,
                             i32, i32, i32, i32, i32, d]
    L.orc_destroy.argtypes = [P]
    L.orc_set_method.argtypes = [P, i32]
    L.orc_info.argtypes = [P, P]
    L.orc_step.argtypes = [P, i64]
    L.orc_check.restype = i32
    L.orc_check.argtypes = [P, d, P]
    L.orc_solve.restype = i32
    L.orc_solve.argtypes = [P, i64, d, P, P, P]
    L.orc_get.argtypes = [P, i32, P, P]
    L.orc_set_point.argtypes = [P, P, P]
    L.orc_kkt.argtypes = [P, i32, P]
    L.orc_gap.restype = d
    L.orc_gap.argtypes = [P, i32, d, P, P]
    L.orc_log_len.restype = i64
    L.orc_log_len.argtypes = [P]
    L.orc_log_copy.argtypes = [P, P]
    L.orc_kkt_at.argtypes = [P, P, P, P]
    L.orc_gap_at.restype = d
    L.orc_gap_at.argtypes = [P, P, P, d, P]
    L.orc_pdhg_map.argtypes = [P, P, P, P, P]
    L.orc_matvec.argtypes = [P, P, P]
    L.orc_matvec_t.argtypes = [P, P, P]
    L.orc_trust_region.restype = d
    L.orc_trust_region.argtypes = [i64, P, P, d, P]
    L.orc_power_iteration.restype = d
    L.orc_power_iteration.argtypes = [i64, i64, P, P, P, i32, d]
    L.orc_transpose.argtypes = [i64, i64, P, P, P, P, P, P, P]
    L.orc_unrolled_grad.restype = d
    L.orc_unrolled_grad.argtypes = [P, i64, P, P, P, P, P]
    L.orc_unrolled_tangent.argtypes = [P, i64, P, P, P, P]
    L.orc_unrolled_value.argtypes = [P, i64, P]
    L.orc_branch_signature.restype = C.c_uint64
    L.orc_branch_signature.argtypes = [P, i64]
    L.orc_restart_iters.restype = i64
    L.orc_restart_iters.argtypes = [P, i64, P, i64]
    L.orc_threads.restype = i32
    L.orc_threads.argtypes = []
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def trust_region(a, d, r):
    """Algorithm 2 on (|g|, distance-to-bound) pairs. Returns (value, lambda)."""
    L = _load()
    a, d = _f64(a), _f64(d)
    lam = np.zeros(1)
    val = L.orc_trust_region(a.size, _p(a), _p(d), float(r), _p(lam))
    return val, float(lam[0])


def power_iteration(lp, iters=1000, tol=1e-10):
    L = _load()
    rp = np.ascontiguousarray(lp.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(lp.col_idx, dtype=np.int32)
    v = _f64(lp.vals)
    return L.orc_power_iteration(lp.m, lp.n, _p(rp), _p(ci), _p(v), iters, tol)


def transpose(m, n, row_ptr, col_idx, vals):
    L = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = _f64(vals)
    nnz = int(rp[-1])
    trp = np.zeros(n + 1, np.int32)
    tci = np.zeros(max(nnz, 1), np.int32)
    tv = np.zeros(max(nnz, 1))
    perm = np.zeros(max(nnz, 1), np.int32)
    L.orc_transpose(m, n, _p(rp), _p(ci), _p(v), _p(trp), _p(tci), _p(tv), _p(perm))
    return trp, tci[:nnz], tv[:nnz], perm[:nnz]


class Oracle:
    """Stateful restarted-PDHG oracle for one LP."""

    def __init__(self, lp, eta=0.0, omega=1.0, beta=float(np.exp(-1.0)),
                 check_period=30, tau0=1, mode=MODE_ADAPTIVE, fixed_len=0,
                 kkt_kind=KKT_RELATIVE, power_iters=1000, power_tol=1e-10,
                 method=METHOD_PDHG, parallel=False):
        # parallel: the OpenMP build (bitwise the same results, all cores)
        L = _load(parallel)
        self._L = L
        self.m, self.n = int(lp.m), int(lp.n)
        self._keep = [np.ascontiguousarray(lp.row_ptr, dtype=np.int32),
                      np.ascontiguousarray(lp.col_idx, dtype=np.int32),
                      _f64(lp.vals), _f64(lp.c), _f64(lp.b), _f64(lp.l),
                      _f64(lp.u),
                      np.ascontiguousarray(lp.row_kind, dtype=np.int8)]
        rp, ci, v, c, b, l, u, k = self._keep
        self.h = L.orc_create(self.m, self.n, _p(rp), _p(ci), _p(v), _p(c),
                              _p(b), _p(l), _p(u), _p(k), float(eta),
                              float(omega), float(beta), int(check_period),
                              int(tau0), int(mode), int(fixed_len),
                              int(kkt_kind), int(power_iters), float(power_tol))
        self.method = int(method)
        L.orc_set_method(self.h, self.method)

    def close(self):
        if self.h:
            self._L.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        out = np.zeros(8)
        self._L.orc_info(self.h, _p(out))
        keys = ["eta", "tau", "sigma", "sigma_max", "k", "t", "restarts",
                "rho_prev"]
        return dict(zip(keys, out.tolist()))

    def step(self, iters):
        self._L.orc_step(self.h, int(iters))

    def check(self, tol=0.0):
        rec = np.zeros(REC)
        conv = self._L.orc_check(self.h, float(tol), _p(rec))
        return bool(conv), rec

    def solve(self, budget, tol):
        res = np.zeros(7)
        x = np.zeros(self.n)
        y = np.zeros(self.m)
        st = self._L.orc_solve(self.h, int(budget), float(tol), _p(res), _p(x), _p(y))
        return dict(status=int(st), k=int(res[1]), restarts=int(res[2]),
                    kkt=res[3], which=int(res[4]), pobj=res[5], dobj=res[6],
                    x=x, y=y)

    def get(self, which=0):
        x = np.zeros(self.n)
        y = np.zeros(self.m)
        self._L.orc_get(self.h, int(which), _p(x), _p(y))
        return x, y

    def set_point(self, x, y):
        x, y = _f64(x), _f64(y)
        self._L.orc_set_point(self.h, _p(x), _p(y))

    def kkt(self, which=0):
        out = np.zeros(7)
        self._L.orc_kkt(self.h, int(which), _p(out))
        return out

    def kkt_at(self, x, y):
        out = np.zeros(7)
        x, y = _f64(x), _f64(y)
        self._L.orc_kkt_at(self.h, _p(x), _p(y), _p(out))
        return out

    def gap(self, which=1, r=-1.0):
        rr = np.zeros(1)
        lam = np.zeros(1)
        v = self._L.orc_gap(self.h, int(which), float(r), _p(rr), _p(lam))
        return v, float(rr[0]), float(lam[0])

    def gap_at(self, x, y, r):
        x, y = _f64(x), _f64(y)
        lam = np.zeros(1)
        v = self._L.orc_gap_at(self.h, _p(x), _p(y), float(r), _p(lam))
        return v, float(lam[0])

    def pdhg_map(self, x, y):
        x, y = _f64(x), _f64(y)
        xo = np.zeros(self.n)
        yo = np.zeros(self.m)
        self._L.orc_pdhg_map(self.h, _p(x), _p(y), _p(xo), _p(yo))
        return xo, yo

    def matvec(self, x):
        x = _f64(x)
        out = np.zeros(self.m)
        self._L.orc_matvec(self.h, _p(x), _p(out))
        return out

    def matvec_t(self, y):
        y = _f64(y)
        out = np.zeros(self.n)
        self._L.orc_matvec_t(self.h, _p(y), _p(out))
        return out

    def unrolled_grad(self, K, x_target):
        """Loss |x_K - x_target|^2 after K unrolled iterations from the
        initial point, and its gradients (c, b, values of A)."""
        xt = _f64(x_target)
        gc, gb = np.zeros(self.n), np.zeros(max(self.m, 1))
        gA = np.zeros(max(int(self._keep[0][-1]), 1))
        xk = np.zeros(self.n)
        loss = self._L.orc_unrolled_grad(self.h, int(K), _p(xt), _p(gc), _p(gb), _p(gA), _p(xk))
        return loss, gc, gb[: self.m], gA[: int(self._keep[0][-1])], xk

    def unrolled_tangent(self, K, dc, db, dA):
        dc, db, dA = _f64(dc), _f64(db if self.m else np.zeros(1)), _f64(dA if len(dA) else np.zeros(1))
        out = np.zeros(self.n)
        self._L.orc_unrolled_tangent(self.h, int(K), _p(dc), _p(db), _p(dA), _p(out))
        return out

    def unrolled_value(self, K):
        out = np.zeros(self.n)
        self._L.orc_unrolled_value(self.h, int(K), _p(out))
        return out

    def branch_signature(self, K):
        return int(self._L.orc_branch_signature(self.h, int(K)))

    def restart_iters(self, K):
        out = np.zeros(4096, np.int64)
        c = self._L.orc_restart_iters(self.h, int(K), _p(out), 4096)
        return out[: min(c, 4096)]

    def log(self):
        n = self._L.orc_log_len(self.h)
        out = np.zeros((max(n, 0), REC))
        if n:
            self._L.orc_log_copy(self.h, _p(out))
        return out


def weight_search(lp, omegas, iters, eta, method=METHOD_PDHG):
    """Primal-weight search of Section 7 (experimental setup; the same
    procedure tunes the extragradient method, appendix on EGM and ADMM):
    the method without restarts for `iters` iterations from the initial
    point at each weight, primal step eta/omega and dual step eta*omega; the
    criterion is
    the KKT error ||(h - Kz)^+||_2 (eq. define:K-and-h-for-lp) of the last
    iterate.  One independent oracle run per weight.  Returns (KKT parts of
    each run as rows [rel, |p|, |d|, pobj, dobj, paper_abs, max_abs], index
    of the smallest paper_abs (NaN as +inf, first on ties), x of each run,
    y of each run)."""
    parts, xs, ys = [], [], []
    for om in omegas:
        o = Oracle(lp, eta=eta, omega=float(om), mode=MODE_NONE, method=method)
        o.step(int(iters))
        parts.append(o.kkt(0))
        x, y = o.get(0)
        xs.append(x)
        ys.append(y)
        o.close()
    parts = np.array(parts)
    crit = np.where(np.isnan(parts[:, 5]), np.inf, parts[:, 5])
    best = int(np.argmin(crit)) if np.isfinite(crit).any() else -1
    return parts, best, np.array(xs), np.array(ys)
