"""ctypes binding of ``libpdhg.so`` (argument marshalling only).

Every computation runs in the HIP kernels of the library; this module moves
arrays into torch device tensors, passes raw pointers and sizes, and turns
return codes into exceptions.  There is no CPU fallback: without the built
library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdhg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pdhg.h")

OK, NOT_CONVERGED = 0, 1
E_INVALID, E_WORKSPACE, E_HIP, E_NUMERICAL = -1, -2, -3, -4
RESTART_NONE, RESTART_ADAPTIVE, RESTART_FLEXIBLE, RESTART_FIXED = 0, 1, 2, 3
KKT_RELATIVE, KKT_PAPER_ABS, KKT_MAX_ABS = 0, 1, 2
METHOD_PDHG, METHOD_EGM = 0, 1
POINT_CURRENT, POINT_AVERAGE, POINT_ANCHOR, POINT_SOLUTION = 0, 1, 2, 3


class PdhgError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


class LP(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("vals", C.c_void_p), ("c", C.c_void_p), ("b", C.c_void_p),
                ("l", C.c_void_p), ("u", C.c_void_p), ("row_kind", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("eta", C.c_double), ("omega", C.c_double), ("beta", C.c_double),
                ("check_period", C.c_int32), ("tau0", C.c_int32),
                ("restart_mode", C.c_int32), ("fixed_len", C.c_int32),
                ("kkt_kind", C.c_int32), ("power_iters", C.c_int32),
                ("power_tol", C.c_double), ("method", C.c_int32)]


class KKT(C.Structure):
    _fields_ = [("kkt", C.c_double), ("kkt_rel", C.c_double),
                ("primal_res", C.c_double), ("dual_res", C.c_double),
                ("pobj", C.c_double), ("dobj", C.c_double),
                ("kkt_paper_abs", C.c_double), ("kkt_max_abs", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("which_point", C.c_int32),
                ("iterations", C.c_int64), ("restarts", C.c_int64),
                ("kkt", C.c_double), ("pobj", C.c_double), ("dobj", C.c_double)]


class Info(C.Structure):
    _fields_ = [("eta", C.c_double), ("tau", C.c_double), ("sigma", C.c_double),
                ("sigma_max", C.c_double), ("k", C.c_int64), ("t", C.c_int64),
                ("restarts", C.c_int64), ("rho_prev", C.c_double),
                ("checks", C.c_int64), ("power_iters_used", C.c_int64),
                ("one_workgroup", C.c_int32), ("bound_classes", C.c_int32)]


class Tune(C.Structure):
    _fields_ = [("slabs_A", C.c_int32), ("slabs_At", C.c_int32),
                ("candidates_A", C.c_int32), ("candidates_At", C.c_int32),
                ("tried_A", C.c_int32 * 4), ("tried_At", C.c_int32 * 4),
                ("ms_A", C.c_double * 4), ("ms_At", C.c_double * 4),
                ("from_cache", C.c_int32), ("reserved", C.c_int32),
                ("lanes_bias_A", C.c_int32), ("lanes_bias_At", C.c_int32),
                ("ms_lanes_A", C.c_double * 3), ("ms_lanes_At", C.c_double * 3),
                ("threads_A", C.c_int32), ("threads_At", C.c_int32),
                ("ms_threads_A", C.c_double * 2), ("ms_threads_At", C.c_double * 2)]


class BatchTune(C.Structure):
    _fields_ = [("placement", C.c_int32), ("index16", C.c_int32),
                ("candidates", C.c_int32), ("reserved", C.c_int32),
                ("tried_placement", C.c_int32 * 4), ("tried_index16", C.c_int32 * 4),
                ("ms", C.c_double * 4)]


class CheckRecord(C.Structure):
    _fields_ = [("v", C.c_double * 14)]


_lib = None


def declared_functions():
    """Names of the functions include/pdhg.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdhg_[a-z_]+)\s*\(", text)))


def load(build_if_missing: bool = True):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError(f"{LIB_PATH} is not built")
        from . import build as _build
        _build.build()
    L = C.CDLL(LIB_PATH)
    P, i32, i64, d, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    L.pdhg_default_params.argtypes = [C.POINTER(Params)]
    L.pdhg_default_params.restype = None
    L.pdhg_workspace_bytes.argtypes = [i64, i64, i64]
    L.pdhg_workspace_bytes.restype = sz
    L.pdhg_create.argtypes = [C.POINTER(LP), C.POINTER(Params), P, sz, P, C.POINTER(P)]
    L.pdhg_create.restype = C.c_int
    L.pdhg_step.argtypes = [P, i64]
    L.pdhg_step.restype = C.c_int
    L.pdhg_restart_check.argtypes = [P, d, C.POINTER(i32), C.POINTER(i32),
                                     C.POINTER(d), C.POINTER(CheckRecord)]
    L.pdhg_restart_check.restype = C.c_int
    L.pdhg_kkt_error.argtypes = [P, i32, C.POINTER(KKT)]
    L.pdhg_kkt_error.restype = C.c_int
    L.pdhg_gap.argtypes = [P, i32, d, C.POINTER(d), C.POINTER(d), C.POINTER(d)]
    L.pdhg_gap.restype = C.c_int
    L.pdhg_solve.argtypes = [P, i64, d, C.POINTER(Result)]
    L.pdhg_solve.restype = C.c_int
    L.pdhg_autotune.argtypes = [P, i32, i32, C.POINTER(Tune)]
    L.pdhg_autotune.restype = C.c_int
    L.pdhg_batch_autotune.argtypes = [P, i32, C.POINTER(BatchTune)]
    L.pdhg_batch_autotune.restype = C.c_int
    L.pdhg_batch_set_schedule.argtypes = [P, i32, i32]
    L.pdhg_batch_set_schedule.restype = C.c_int
    L.pdhg_solve_many_workspace_bytes.argtypes = [i32]
    L.pdhg_solve_many_workspace_bytes.restype = sz
    L.pdhg_solve_many.argtypes = [P, i32, i64, d, P, sz, P]
    L.pdhg_solve_many.restype = C.c_int
    L.pdhg_get_iterate.argtypes = [P, i32, P, P]
    L.pdhg_get_iterate.restype = C.c_int
    L.pdhg_set_iterate.argtypes = [P, P, P]
    L.pdhg_set_iterate.restype = C.c_int
    L.pdhg_set_schedule.argtypes = [P, i32, i32, i32, i32]
    L.pdhg_set_schedule.restype = C.c_int
    L.pdhg_state_bytes.argtypes = [P]
    L.pdhg_state_bytes.restype = C.c_size_t
    L.pdhg_get_state.argtypes = [P, P, C.c_size_t]
    L.pdhg_get_state.restype = C.c_int
    L.pdhg_set_state.argtypes = [P, P, C.c_size_t]
    L.pdhg_set_state.restype = C.c_int
    L.pdhg_get_info.argtypes = [P, C.POINTER(Info)]
    L.pdhg_get_info.restype = C.c_int
    L.pdhg_get_check_log.argtypes = [P, P, i64, C.POINTER(i64)]
    L.pdhg_get_check_log.restype = C.c_int
    L.pdhg_matvec.argtypes = [P, i32, P, P]
    L.pdhg_matvec.restype = C.c_int
    L.pdhg_get_transpose.argtypes = [P, P, P, P, P]
    L.pdhg_get_transpose.restype = C.c_int
    L.pdhg_time_iterations.argtypes = [P, i64, C.POINTER(d), C.POINTER(d)]
    L.pdhg_time_iterations.restype = C.c_int
    L.pdhg_weight_search_workspace_bytes.argtypes = [i64, i64, i32]
    L.pdhg_weight_search_workspace_bytes.restype = sz
    L.pdhg_weight_search.argtypes = [P, P, i32, i64, P, sz, P, C.POINTER(i32), P, P]
    L.pdhg_weight_search.restype = C.c_int
    L.pdhg_set_primal_weight.argtypes = [P, d]
    L.pdhg_set_primal_weight.restype = C.c_int
    L.pdhg_destroy.argtypes = [P]
    L.pdhg_destroy.restype = None
    L.pdhg_trust_region_workspace_bytes.argtypes = [i64]
    L.pdhg_trust_region_workspace_bytes.restype = sz
    L.pdhg_linear_trust_region.argtypes = [i64, P, P, d, P, sz, P, C.POINTER(d), C.POINTER(d)]
    L.pdhg_linear_trust_region.restype = C.c_int
    L.pdhg_time_copy.argtypes = [P, P, i64, i32, P, C.POINTER(d)]
    L.pdhg_time_copy.restype = C.c_int
    L.pdhg_time_gather.argtypes = [P, P, P, P, i64, i32, P, C.POINTER(d)]
    L.pdhg_time_gather.restype = C.c_int
    L.pdhg_gather_only_outputs.argtypes = [i64]
    L.pdhg_gather_only_outputs.restype = i64
    L.pdhg_time_gather_only.argtypes = [P, i64, P, i64, P, i32, P, C.POINTER(d)]
    L.pdhg_time_gather_only.restype = C.c_int
    L.pdhg_linear_trust_region_static.argtypes = [i64, P, P, d, P, C.POINTER(d), C.POINTER(d)]
    L.pdhg_linear_trust_region_static.restype = C.c_int
    L.pdhg_batch_workspace_bytes.argtypes = [i32, P, P, P]
    L.pdhg_batch_workspace_bytes.restype = sz
    L.pdhg_batch_create.argtypes = [i32, P, P, P, sz, P, C.POINTER(P)]
    L.pdhg_batch_create.restype = C.c_int
    L.pdhg_batch_step.argtypes = [P, i64]
    L.pdhg_batch_step.restype = C.c_int
    L.pdhg_batch_solve.argtypes = [P, i64, d, P]
    L.pdhg_batch_solve.restype = C.c_int
    L.pdhg_batch_get_iterate.argtypes = [P, i32, i32, P, P]
    L.pdhg_batch_get_iterate.restype = C.c_int
    L.pdhg_batch_get_info.argtypes = [P, i32, C.POINTER(Info)]
    L.pdhg_batch_get_info.restype = C.c_int
    L.pdhg_batch_get_check_log.argtypes = [P, i32, P, i64, C.POINTER(i64)]
    L.pdhg_batch_get_check_log.restype = C.c_int
    L.pdhg_batch_set_data.argtypes = [P, P, P, P]
    L.pdhg_batch_set_data.restype = C.c_int
    L.pdhg_batch_tape_bytes.argtypes = [P, i64]
    L.pdhg_batch_tape_bytes.restype = sz
    L.pdhg_batch_unrolled_forward.argtypes = [P, i64, P, sz, P]
    L.pdhg_batch_unrolled_forward.restype = C.c_int
    L.pdhg_batch_unrolled_backward.argtypes = [P, i64, P, sz, P, P, P, P]
    L.pdhg_batch_unrolled_backward.restype = C.c_int
    L.pdhg_batch_destroy.argtypes = [P]
    L.pdhg_batch_destroy.restype = None
    L.pdhg_strerror.argtypes = [C.c_int]
    L.pdhg_strerror.restype = C.c_char_p
    _lib = L
    return L


def strerror(code: int) -> str:
    return load().pdhg_strerror(int(code)).decode()


def default_params() -> Params:
    p = Params()
    load().pdhg_default_params(C.byref(p))
    return p


def workspace_bytes(m: int, n: int, nnz: int) -> int:
    return int(load().pdhg_workspace_bytes(m, n, nnz))


def _check(rc, where, allow=(OK,)):
    if rc not in allow:
        raise PdhgError(rc, where)
    return rc


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def _dev_workspace(nbytes, device):
    import torch
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf[off:off + int(nbytes)]


class Solver:
    """One LP on one GPU: a handle of the C library plus the torch tensors
    that own its device memory (problem data and workspace)."""

    def __init__(self, lp, eta=0.0, omega=1.0, beta=float(np.exp(-1.0)),
                 check_period=30, tau0=1, restart_mode=RESTART_ADAPTIVE,
                 fixed_len=0, kkt_kind=KKT_RELATIVE, power_iters=1000,
                 power_tol=1e-10, device="cuda:0", stream=None, method=METHOD_PDHG):
        import torch
        L = load()
        self._L = L
        self.device = torch.device(device)
        self.stream = stream
        self.m, self.n = int(lp.m), int(lp.n)
        dev = self.device
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).to(dev)
        self.row_ptr = i32(lp.row_ptr)
        self.nnz = int(np.asarray(lp.row_ptr)[-1]) if self.m >= 0 else 0
        self.col_idx = i32(lp.col_idx) if self.nnz else torch.zeros(1, dtype=torch.int32, device=dev)
        self.vals = f64(lp.vals) if self.nnz else torch.zeros(1, dtype=torch.float64, device=dev)
        self.c, self.l, self.u = f64(lp.c), f64(lp.l), f64(lp.u)
        self.b = f64(lp.b) if self.m else torch.zeros(1, dtype=torch.float64, device=dev)
        rk = getattr(lp, "row_kind", None)
        self.row_kind = (torch.as_tensor(np.ascontiguousarray(rk, dtype=np.int8)).to(dev)
                         if rk is not None and self.m else None)
        self._lp = LP(self.m, self.n, self.nnz, self.row_ptr.data_ptr(),
                      self.col_idx.data_ptr(), self.vals.data_ptr(), self.c.data_ptr(),
                      self.b.data_ptr(), self.l.data_ptr(), self.u.data_ptr(),
                      self.row_kind.data_ptr() if self.row_kind is not None else None)
        self.params = Params(float(eta), float(omega), float(beta), int(check_period),
                             int(tau0), int(restart_mode), int(fixed_len), int(kkt_kind),
                             int(power_iters), float(power_tol), int(method))
        nbytes = L.pdhg_workspace_bytes(self.m, self.n, self.nnz)
        if nbytes == 0:
            raise PdhgError(E_INVALID, "pdhg_workspace_bytes")
        self._ws_owner, self.workspace = _dev_workspace(nbytes, dev)
        h = C.c_void_p()
        rc = L.pdhg_create(C.byref(self._lp), C.byref(self.params),
                           _ptr(self.workspace), nbytes, _stream_handle(stream), C.byref(h))
        _check(rc, "pdhg_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self._L.pdhg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- iteration -------------------------------------------------------
    def step(self, iters):
        _check(self._L.pdhg_step(self.h, int(iters)), "pdhg_step")

    def check(self, tol=0.0):
        conv, rst = C.c_int32(), C.c_int32()
        rho = C.c_double()
        rec = CheckRecord()
        _check(self._L.pdhg_restart_check(self.h, float(tol), C.byref(conv), C.byref(rst),
                                          C.byref(rho), C.byref(rec)), "pdhg_restart_check")
        return bool(conv.value), np.array(rec.v[:])

    def solve(self, max_iters, tol):
        res = Result()
        rc = self._L.pdhg_solve(self.h, int(max_iters), float(tol), C.byref(res))
        _check(rc, "pdhg_solve", allow=(OK, NOT_CONVERGED))
        return dict(status=int(res.status), k=int(res.iterations), restarts=int(res.restarts),
                    kkt=float(res.kkt), which=int(res.which_point), pobj=float(res.pobj),
                    dobj=float(res.dobj))

    def autotune(self, iters=20, use_cache=True):
        """pdhg_autotune: time the column-slab counts of A x and A'y on this
        matrix, then the lanes per row (one power of two below, at and above
        the rule), then the threads per workgroup (256 or 128), keeping the
        fastest of each; returns the choices in use and the timings (ms per
        product) of the candidates tried."""
        t = Tune()
        _check(self._L.pdhg_autotune(self.h, int(iters), 1 if use_cache else 0, C.byref(t)),
               "pdhg_autotune")
        cached = bool(t.from_cache)
        return dict(slabs_A=t.slabs_A, slabs_At=t.slabs_At, from_cache=cached,
                    lanes_bias_A=t.lanes_bias_A, lanes_bias_At=t.lanes_bias_At,
                    A={int(t.tried_A[i]): float(t.ms_A[i]) for i in range(t.candidates_A)},
                    At={int(t.tried_At[i]): float(t.ms_At[i]) for i in range(t.candidates_At)},
                    lanes_A={} if cached else {b - 1: float(t.ms_lanes_A[b]) for b in range(3)},
                    lanes_At={} if cached else {b - 1: float(t.ms_lanes_At[b])
                                                for b in range(3)},
                    threads_A=t.threads_A, threads_At=t.threads_At,
                    ms_threads_A={} if cached else {256: float(t.ms_threads_A[0]),
                                                    128: float(t.ms_threads_A[1])},
                    ms_threads_At={} if cached else {256: float(t.ms_threads_At[0]),
                                                     128: float(t.ms_threads_At[1])})

    def set_schedule(self, slabs_A=1, slabs_At=1, lanes_bias_A=0, lanes_bias_At=0):
        """pdhg_set_schedule: pin the slab counts and lanes-per-row biases."""
        _check(self._L.pdhg_set_schedule(self.h, int(slabs_A), int(slabs_At), int(lanes_bias_A),
                                         int(lanes_bias_At)), "pdhg_set_schedule")

    # -- evaluation --------------------------------------------------------
    def kkt(self, which=POINT_CURRENT):
        out = KKT()
        _check(self._L.pdhg_kkt_error(self.h, int(which), C.byref(out)), "pdhg_kkt_error")
        return {k: getattr(out, k) for k, _ in KKT._fields_}

    def gap(self, which=POINT_AVERAGE, r=-1.0):
        rho, rr, lam = C.c_double(), C.c_double(), C.c_double()
        _check(self._L.pdhg_gap(self.h, int(which), float(r), C.byref(rho), C.byref(rr),
                                C.byref(lam)), "pdhg_gap")
        return rho.value, rr.value, lam.value

    def get_iterate(self, which=POINT_CURRENT):
        import torch
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        y = torch.empty(max(self.m, 1), dtype=torch.float64, device=self.device)
        _check(self._L.pdhg_get_iterate(self.h, int(which), _ptr(x), _ptr(y)),
               "pdhg_get_iterate")
        return x, y[: self.m]

    # -- checkpoint ------------------------------------------------------
    def state_bytes(self):
        return int(self._L.pdhg_state_bytes(self.h))

    def get_state(self):
        """The handle's solver state as a device byte tensor (opaque)."""
        nbytes = self.state_bytes()
        owner, view = _dev_workspace(nbytes, self.device)
        _check(self._L.pdhg_get_state(self.h, _ptr(view), nbytes), "pdhg_get_state")
        return (owner, view)

    def set_state(self, state):
        owner, view = state
        _check(self._L.pdhg_set_state(self.h, _ptr(view), int(view.numel())), "pdhg_set_state")

    def set_iterate(self, x, y):
        import torch
        x = torch.as_tensor(x, dtype=torch.float64).to(self.device).contiguous()
        y = torch.as_tensor(y, dtype=torch.float64).to(self.device).contiguous()
        if self.m == 0:
            y = torch.zeros(1, dtype=torch.float64, device=self.device)
        self._keep_point = (x, y)
        _check(self._L.pdhg_set_iterate(self.h, _ptr(x), _ptr(y)), "pdhg_set_iterate")

    def info(self):
        out = Info()
        _check(self._L.pdhg_get_info(self.h, C.byref(out)), "pdhg_get_info")
        return {k: getattr(out, k) for k, _ in Info._fields_}

    def check_log(self, max_records=4096):
        arr = (CheckRecord * max_records)()
        cnt = C.c_int64()
        _check(self._L.pdhg_get_check_log(self.h, C.cast(arr, C.c_void_p), max_records,
                                          C.byref(cnt)), "pdhg_get_check_log")
        return np.array([arr[i].v[:] for i in range(cnt.value)]).reshape(-1, 14)

    def matvec(self, v, transpose=False):
        import torch
        v = torch.as_tensor(v, dtype=torch.float64).to(self.device).contiguous()
        out = torch.empty(self.n if transpose else max(self.m, 1), dtype=torch.float64,
                          device=self.device)
        _check(self._L.pdhg_matvec(self.h, 1 if transpose else 0, _ptr(v), _ptr(out)),
               "pdhg_matvec")
        return out if transpose else out[: self.m]

    def time_iterations(self, iters):
        """Mean kernel milliseconds (primal, dual) over `iters` iterations."""
        a, b = C.c_double(), C.c_double()
        _check(self._L.pdhg_time_iterations(self.h, int(iters), C.byref(a), C.byref(b)),
               "pdhg_time_iterations")
        return a.value, b.value

    # -- primal weight (Section 7) ---------------------------------------
    def weight_search(self, omegas, iters=5000, want_iterates=False):
        """Non-restarted PDHG for `iters` iterations at every weight in
        `omegas` (one pass over A or A' per product for all of them).
        Returns (list of KKT dicts, index of the smallest kkt_paper_abs,
        x [count, n] and y [count, m] tensors or None)."""
        import torch
        om = np.ascontiguousarray(omegas, dtype=np.float64)
        cnt = int(om.size)
        nbytes = self._L.pdhg_weight_search_workspace_bytes(self.m, self.n, cnt)
        if nbytes == 0:
            raise PdhgError(E_INVALID, "pdhg_weight_search_workspace_bytes")
        _own, ws = _dev_workspace(nbytes, self.device)
        kk = (KKT * cnt)()
        best = C.c_int32()
        x = y = None
        if want_iterates:
            x = torch.empty(cnt * self.n, dtype=torch.float64, device=self.device)
            y = torch.empty(max(cnt * self.m, 1), dtype=torch.float64, device=self.device)
        rc = self._L.pdhg_weight_search(
            self.h, om.ctypes.data_as(C.c_void_p), cnt, int(iters), _ptr(ws), nbytes,
            C.cast(kk, C.c_void_p), C.byref(best), _ptr(x) if x is not None else None,
            _ptr(y) if y is not None else None)
        _check(rc, "pdhg_weight_search")
        out = [{k: getattr(kk[w], k) for k, _ in KKT._fields_} for w in range(cnt)]
        if want_iterates:
            x = x.view(cnt, self.n)
            y = y[: cnt * self.m].view(cnt, self.m)
        return out, int(best.value), x, y

    def set_primal_weight(self, omega):
        _check(self._L.pdhg_set_primal_weight(self.h, float(omega)), "pdhg_set_primal_weight")

    def transpose_csr(self):
        import torch
        dev = self.device
        trp = torch.empty(self.n + 1, dtype=torch.int32, device=dev)
        tci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        tv = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev)
        perm = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        _check(self._L.pdhg_get_transpose(self.h, _ptr(trp), _ptr(tci), _ptr(tv), _ptr(perm)),
               "pdhg_get_transpose")
        k = self.nnz
        return trp, tci[:k], tv[:k], perm[:k]


class _DeviceLP:
    """Device tensors of one LP and its C struct."""

    def __init__(self, lp, dev):
        import torch
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).to(dev)
        self.m, self.n = int(lp.m), int(lp.n)
        self.nnz = int(np.asarray(lp.row_ptr)[-1])
        self.row_ptr = i32(lp.row_ptr)
        self.col_idx = i32(lp.col_idx) if self.nnz else torch.zeros(1, dtype=torch.int32, device=dev)
        self.vals = f64(lp.vals) if self.nnz else torch.zeros(1, dtype=torch.float64, device=dev)
        self.c, self.l, self.u = f64(lp.c), f64(lp.l), f64(lp.u)
        self.b = f64(lp.b) if self.m else torch.zeros(1, dtype=torch.float64, device=dev)
        rk = getattr(lp, "row_kind", None)
        self.row_kind = (torch.as_tensor(np.ascontiguousarray(rk, dtype=np.int8)).to(dev)
                         if rk is not None and self.m else None)
        self.struct = LP(self.m, self.n, self.nnz, self.row_ptr.data_ptr(),
                         self.col_idx.data_ptr(), self.vals.data_ptr(), self.c.data_ptr(),
                         self.b.data_ptr(), self.l.data_ptr(), self.u.data_ptr(),
                         self.row_kind.data_ptr() if self.row_kind is not None else None)


def _result_dict(r):
    return dict(status=int(r.status), k=int(r.iterations), restarts=int(r.restarts),
                kkt=float(r.kkt), which=int(r.which_point), pobj=float(r.pobj),
                dobj=float(r.dobj))


def solve_many(solvers, max_iters, tol):
    """pdhg_solve_many on several Solver handles at once: the ones on the
    one-workgroup path run together, one workgroup per LP.  Returns one
    result dict per solver, as Solver.solve does."""
    import torch
    solvers = list(solvers)
    if not solvers:
        return []
    L = solvers[0]._L
    n = len(solvers)
    hs = (C.c_void_p * n)(*[s.h for s in solvers])
    nbytes = int(L.pdhg_solve_many_workspace_bytes(n))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=solvers[0].device)
    res = (Result * n)()
    rc = L.pdhg_solve_many(C.cast(hs, C.c_void_p), n, int(max_iters), float(tol), _ptr(ws),
                           nbytes, C.cast(res, C.c_void_p))
    _check(rc, "pdhg_solve_many", allow=(OK, NOT_CONVERGED))
    return [_result_dict(r) for r in res]


class BatchSolver:
    """Many independent LPs solved by the same launches (pdhg_batch_*)."""

    def __init__(self, lps, params=None, device="cuda:0", stream=None, **common):
        import torch
        L = load()
        self._L = L
        self.device = torch.device(device)
        self.lps = [_DeviceLP(lp, self.device) for lp in lps]
        self.count = len(self.lps)
        arr = (LP * self.count)(*[d.struct for d in self.lps])
        if params is None:
            params = [{}] * self.count
        elif isinstance(params, dict):
            params = [params] * self.count
        prm = (Params * self.count)()
        for i, p in enumerate(params):
            q = dict(eta=0.0, omega=1.0, beta=float(np.exp(-1.0)), check_period=30, tau0=1,
                     restart_mode=RESTART_ADAPTIVE, fixed_len=0, kkt_kind=KKT_RELATIVE,
                     power_iters=1000, power_tol=1e-10)
            q.update(common)
            q.update(p)
            prm[i] = Params(float(q["eta"]), float(q["omega"]), float(q["beta"]),
                            int(q["check_period"]), int(q["tau0"]), int(q["restart_mode"]),
                            int(q["fixed_len"]), int(q["kkt_kind"]), int(q["power_iters"]),
                            float(q["power_tol"]))
        ms = np.array([d.m for d in self.lps], np.int64)
        ns = np.array([d.n for d in self.lps], np.int64)
        zs = np.array([d.nnz for d in self.lps], np.int64)
        nbytes = L.pdhg_batch_workspace_bytes(self.count, ms.ctypes.data, ns.ctypes.data,
                                              zs.ctypes.data)
        if nbytes == 0:
            raise PdhgError(E_INVALID, "pdhg_batch_workspace_bytes")
        self._ws_owner, self.workspace = _dev_workspace(nbytes, self.device)
        h = C.c_void_p()
        rc = L.pdhg_batch_create(self.count, C.cast(arr, C.c_void_p), C.cast(prm, C.c_void_p),
                                 _ptr(self.workspace), nbytes, _stream_handle(stream), C.byref(h))
        _check(rc, "pdhg_batch_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self._L.pdhg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, iters):
        _check(self._L.pdhg_batch_step(self.h, int(iters)), "pdhg_batch_step")

    def solve(self, max_iters, tol):
        res = (Result * self.count)()
        rc = self._L.pdhg_batch_solve(self.h, int(max_iters), float(tol), C.cast(res, C.c_void_p))
        _check(rc, "pdhg_batch_solve", allow=(OK, NOT_CONVERGED))
        return [dict(status=int(r.status), k=int(r.iterations), restarts=int(r.restarts),
                     kkt=float(r.kkt), which=int(r.which_point), pobj=float(r.pobj),
                     dobj=float(r.dobj)) for r in res]

    def get_iterate(self, index, which=POINT_CURRENT):
        import torch
        d = self.lps[index]
        x = torch.empty(d.n, dtype=torch.float64, device=self.device)
        y = torch.empty(max(d.m, 1), dtype=torch.float64, device=self.device)
        _check(self._L.pdhg_batch_get_iterate(self.h, int(index), int(which), _ptr(x), _ptr(y)),
               "pdhg_batch_get_iterate")
        return x, y[: d.m]

    def info(self, index):
        out = Info()
        _check(self._L.pdhg_batch_get_info(self.h, int(index), C.byref(out)),
               "pdhg_batch_get_info")
        return {k: getattr(out, k) for k, _ in Info._fields_}

    def autotune(self, iters=20):
        """pdhg_batch_autotune: time the SpMV schedules (XCD placement or
        row order; 16-bit or 32-bit indices) and keep the fastest; returns
        the schedule in use and {(placement, index16): ms per pair of
        products}."""
        t = BatchTune()
        _check(self._L.pdhg_batch_autotune(self.h, int(iters), C.byref(t)),
               "pdhg_batch_autotune")
        return dict(placement=t.placement, index16=t.index16,
                    ms={(int(t.tried_placement[i]), int(t.tried_index16[i])): float(t.ms[i])
                        for i in range(t.candidates)})

    def set_schedule(self, placement, index16):
        _check(self._L.pdhg_batch_set_schedule(self.h, int(placement), int(index16)),
               "pdhg_batch_set_schedule")

    # -- differentiation -------------------------------------------------
    @property
    def sizes(self):
        return ([d.n for d in self.lps], [d.m for d in self.lps], [d.nnz for d in self.lps])

    def concat_data(self):
        """(c, b, vals) of the whole batch as concatenated device tensors."""
        import torch
        c = torch.cat([d.c for d in self.lps])
        b = torch.cat([d.b[: d.m] for d in self.lps])
        v = torch.cat([d.vals[: d.nnz] for d in self.lps])
        return c, b, v

    def set_data(self, c, b, vals):
        import torch
        c = c.detach().to(self.device, torch.float64).contiguous()
        b = b.detach().to(self.device, torch.float64).contiguous()
        vals = vals.detach().to(self.device, torch.float64).contiguous()
        self._data_keep = (c, b, vals)
        _check(self._L.pdhg_batch_set_data(self.h, _ptr(c), _ptr(b), _ptr(vals)),
               "pdhg_batch_set_data")

    def unrolled_forward(self, K):
        """x_K (concatenated) after K unrolled iterations from the initial
        points, and the tape the backward pass needs."""
        import torch
        nbytes = self._L.pdhg_batch_tape_bytes(self.h, int(K))
        if nbytes == 0:
            raise PdhgError(E_INVALID, "pdhg_batch_tape_bytes")
        owner, tape = _dev_workspace(nbytes, self.device)
        N = sum(d.n for d in self.lps)
        xk = torch.empty(N, dtype=torch.float64, device=self.device)
        _check(self._L.pdhg_batch_unrolled_forward(self.h, int(K), _ptr(tape), nbytes, _ptr(xk)),
               "pdhg_batch_unrolled_forward")
        return xk, (owner, tape, nbytes, int(K))

    def unrolled_backward(self, tape, dL_dxK):
        import torch
        owner, buf, nbytes, K = tape
        N = sum(d.n for d in self.lps)
        M = sum(d.m for d in self.lps)
        Z = sum(d.nnz for d in self.lps)
        g = dL_dxK.detach().to(self.device, torch.float64).contiguous()
        gc = torch.empty(N, dtype=torch.float64, device=self.device)
        gb = torch.empty(max(M, 1), dtype=torch.float64, device=self.device)
        gA = torch.empty(max(Z, 1), dtype=torch.float64, device=self.device)
        _check(self._L.pdhg_batch_unrolled_backward(self.h, K, _ptr(buf), nbytes, _ptr(g),
                                                    _ptr(gc), _ptr(gb), _ptr(gA)),
               "pdhg_batch_unrolled_backward")
        return gc, gb[:M], gA[:Z]

    def check_log(self, index, max_records=512):
        arr = (CheckRecord * max_records)()
        cnt = C.c_int64()
        _check(self._L.pdhg_batch_get_check_log(self.h, int(index), C.cast(arr, C.c_void_p),
                                                max_records, C.byref(cnt)),
               "pdhg_batch_get_check_log")
        return np.array([arr[i].v[:] for i in range(cnt.value)]).reshape(-1, 14)


def _make_unrolled():
    import torch

    class PDHGUnrolled(torch.autograd.Function):
        """x_K of K unrolled restarted-PDHG iterations for every LP of a
        BatchSolver, differentiable in the concatenated (c, b, values of A).
        Restart decisions and projection masks are those of the forward
        pass; step sizes are constants."""

        @staticmethod
        def forward(ctx, c, b, vals, solver, K):
            solver.set_data(c, b, vals)
            xk, tape = solver.unrolled_forward(K)
            ctx.solver = solver
            ctx.tape = tape
            return xk

        @staticmethod
        def backward(ctx, grad_xk):
            gc, gb, gA = ctx.solver.unrolled_backward(ctx.tape, grad_xk)
            return gc, gb, gA, None, None

    return PDHGUnrolled


_UNROLLED = None


def pdhg_unrolled(c, b, vals, solver, K):
    """Differentiable x_K (see PDHGUnrolled)."""
    global _UNROLLED
    if _UNROLLED is None:
        _UNROLLED = _make_unrolled()
    return _UNROLLED.apply(c, b, vals, solver, K)


def time_copy(src, dst, reps=20, stream=None):
    """Mean ms of the library's streaming copy dst = src (device float64
    tensors of equal size)."""
    L = load()
    ms = C.c_double()
    _check(L.pdhg_time_copy(_ptr(src), _ptr(dst), int(src.numel()), int(reps),
                            _stream_handle(stream), C.byref(ms)), "pdhg_time_copy")
    return ms.value


def time_gather(idx, val, x, out, reps=20, stream=None):
    """Mean ms of the library's plain gather out = val * x[idx]."""
    L = load()
    ms = C.c_double()
    _check(L.pdhg_time_gather(_ptr(idx), _ptr(val), _ptr(x), _ptr(out), int(idx.numel()),
                              int(reps), _stream_handle(stream), C.byref(ms)),
           "pdhg_time_gather")
    return ms.value


def time_gather_only(x, n, idx=None, reps=20, stream=None):
    """Mean ms of the library's gathers alone: n gathers of x at idx (a
    device int32 tensor of n indices) or, with idx None, at hashed indices
    over all of x (its length a power of two).  Returns (ms, out)."""
    import torch
    L = load()
    nout = int(L.pdhg_gather_only_outputs(int(n)))
    if nout < 1:
        raise PdhgError(E_INVALID, "pdhg_gather_only_outputs")
    out = torch.empty(nout, dtype=torch.float64, device=x.device)
    ms = C.c_double()
    _check(L.pdhg_time_gather_only(None if idx is None else _ptr(idx), int(n), _ptr(x),
                                   int(x.numel()), _ptr(out), int(reps), _stream_handle(stream),
                                   C.byref(ms)), "pdhg_time_gather_only")
    return ms.value, out


TR_STATIC_MAX_N = 262144


def linear_trust_region_static(a, d, r, device="cuda:0", stream=None):
    """The same trust region through pdhg_linear_trust_region_static (no
    workspace: the library's static scratch); returns (value, lambda)."""
    import torch
    L = load()
    a = torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
    d = torch.as_tensor(d, dtype=torch.float64).to(device).contiguous()
    N = int(a.numel())
    val, lam = C.c_double(), C.c_double()
    rc = L.pdhg_linear_trust_region_static(N, _ptr(a) if N else None, _ptr(d) if N else None,
                                           float(r), _stream_handle(stream), C.byref(val),
                                           C.byref(lam))
    _check(rc, "pdhg_linear_trust_region_static")
    return val.value, lam.value


def linear_trust_region(a, d, r, device="cuda:0", stream=None):
    """Stand-alone trust region on device tensors (or arrays): returns
    (value, lambda)."""
    import torch
    L = load()
    a = torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
    d = torch.as_tensor(d, dtype=torch.float64).to(device).contiguous()
    N = int(a.numel())
    nbytes = L.pdhg_trust_region_workspace_bytes(N)
    owner, ws = _dev_workspace(nbytes, device)
    val, lam = C.c_double(), C.c_double()
    rc = L.pdhg_linear_trust_region(N, _ptr(a) if N else None, _ptr(d) if N else None,
                                    float(r), _ptr(ws), nbytes, _stream_handle(stream),
                                    C.byref(val), C.byref(lam))
    _check(rc, "pdhg_linear_trust_region")
    del owner
    return val.value, lam.value
