#!/usr/bin/env python3
"""Throughput of restarted PDHG on one MI355X.

One step = one block of the solve loop: `check_period` (30) PDHG iterations
(A'y and A x+ SpMVs with fused projections and running sums) followed by
the restart check (check-time SpMVs, KKT at z and z-bar, the normalized
duality gap by the trust-region bisection, restart decision and restart).
The timed region replays K blocks through pdhg_solve with tol = 0, so no
block is skipped.  `value` is PDHG iterations per second with the LP
already resident in HBM.

Default workload: the large sparse LP, 1,000,000 x 2,000,000 with power-law
column counts (exponent 2, 1..1000 per column, ~9.1M entries), random-sign
log-uniform values in [1e-3, 1e3], planted optimum, seed 3.

The roofline figure is for the dominant half-step (A'y with the primal
update, or A x+ with the dual update), timed with HIP events on the
handle's stream right after the timed region.  A half-step is one SpMV
kernel with the update fused, or, where the gathered vector is split into
column slabs, one launch per slab, the last adding up the slabs' row sums
and applying the update.  Algorithmic bytes per half-step are
    primal: 12 nnz + 60 n + 8 m     dual: 12 nnz + 61 m + 8 n
(values + int32 indices of A' or A, row pointers, the vector reads and
writes of the epilogue, and one compulsory read of the gathered vector).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PDHG iter/s + HBM GB/s; time to 1e-8 rel KKT, batched vs plain"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2105_12715_amd import lpgen
    if name == "large":
        return lpgen.large_powerlaw(3), "large power-law LP 1,000,000 x 2,000,000 (seed 3)"
    if name == "medium":
        return lpgen.medium(2), "medium LP 20,000 x 50,000, 10 per column (seed 2)"
    if name == "small":
        return lpgen.small_dense(1), "small LP 50 x 100, Bernoulli(0.1) (seed 1)"
    raise SystemExit(f"unknown workload {name}")


def halfstep_bytes(m, n, nnz):
    """Algorithmic bytes of one primal and one dual half-step, from the
    byte model of the path.  Both stream their matrix (8-byte value and
    4-byte index per entry) and row pointers (4 bytes per row) and read the
    gathered vector once (8 bytes per element).  Primal, per column: x, c,
    l, u and S_x reads, x and S_x writes (56).  Dual, per row: y, b, q,
    S_y and row-kind reads, y, S_y and q writes (57).  The kernels move
    less than this where they can: a class byte per column instead of l and
    u when the bounds take at most four pairs, and the running sums read and
    written every other iteration.  The measured traffic is reported next
    to it."""
    return 12 * nnz + 60 * n + 8 * m, 12 * nnz + 61 * m + 8 * n


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("pdhg_kernels.hip", "pdhg_device.h", "pdhg_internal.h"):
        with open(os.path.join(ROOT, "paper_2105_12715_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken with the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(lp, eta, budget_s=12.0):
    """The oracle on the same LP and schedule (whole blocks of 30 iterations
    with their restart checks), timed on the host: the plain build on one
    core, and the OpenMP build of the same source (bitwise the same
    iterates) on every core the process may use.  About budget_s seconds
    of CPU work each."""
    import oracle

    def timed(parallel, budget):
        o = oracle.Oracle(lp, eta=eta, mode=oracle.MODE_ADAPTIVE, parallel=parallel)
        # calibrate on 2 iterations, then whole blocks for about `budget`
        t0 = time.perf_counter()
        o.step(2)
        per_iter = (time.perf_counter() - t0) / 2
        blocks = max(1, int(budget / (per_iter * 30 * 1.5)))
        o.close()
        o2 = oracle.Oracle(lp, eta=eta, mode=oracle.MODE_ADAPTIVE, parallel=parallel)
        t0 = time.perf_counter()
        o2.solve(30 * blocks, 0.0)
        dt = time.perf_counter() - t0
        o2.close()
        return 30 * blocks / dt, blocks, dt

    v1, b1, d1 = timed(False, budget_s)
    cores = oracle.threads(parallel=True)
    vp, bp, dp = timed(True, budget_s)
    par = {"value": vp, "unit": "iter/s", "cores": cores,
           "sample": f"{bp} block(s) of 30 iterations + restart check on the same LP, FP64 C "
                     f"oracle built with OpenMP (bitwise the plain build's iterates), "
                     f"{cores} threads, {dp:.1f} s"}
    one = {"value": v1, "unit": "iter/s", "cores": 1,
           "sample": f"{b1} block(s) of 30 iterations + restart check on the same LP, plain "
                     f"single-threaded FP64 C oracle, {d1:.1f} s"}
    # the faster of the two builds is the baseline (threads do not pay off
    # on a small LP); the other stands beside it
    best, other = (par, one) if vp >= v1 else (one, par)
    return {**best, "kind": "oracle", "other_build": other}


def run_batch(args):
    """Batched versus sequential time to relative KKT <= tol on the uneven
    batch: 256 planted LPs, m_i ~ U{200..20000}, n_i = 2 m_i, 5 per column,
    bounds [0,1].  The batch runs until every LP has converged (or the
    budget ends), printing progress per chunk.  Each LP of a batch follows
    exactly the iterates of its own single-LP solve (a GPU test checks
    this), so the sequential time is the sum over LPs of its iteration
    count times the measured per-iteration time of its single-LP solve.

    The model is checked on the three LPs with the fewest iterations (each
    solved alone to the tolerance) and on the three with the most (each
    timed alone over a truncated budget).  The time to tolerance is also
    reported for the converged subset alone: the batch's clock when its
    last member converged (interpolated inside the chunk) against the sum
    of the subset's sequential times.  One member that does not converge
    is run by the oracle for its first --oracle-iters iterations beside
    its own GPU solve, check by check, to show whether its stall is the
    method's or a discrepancy of the GPU path."""
    import numpy as np
    import torch
    from paper_2105_12715_amd import _lib, lpgen

    t0 = time.perf_counter()
    lps = [lpgen.batch_member(i) for i in range(args.batch_count)]
    log(f"{len(lps)} LPs generated in {time.perf_counter() - t0:.1f}s: sum m "
        f"{sum(lp.m for lp in lps)}, sum nnz {sum(lp.nnz for lp in lps)}")
    t0 = time.perf_counter()
    b = _lib.BatchSolver(lps)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    log(f"batch setup (validation, transposes, 256 power iterations) {setup:.2f}s")
    tol = args.tol
    t0 = time.perf_counter()
    done_k = 0
    res = None
    clock = [(0, 0.0)]  # (batch iterations, seconds) after every chunk
    while done_k < args.budget:
        chunk = min(args.chunk, args.budget - done_k)
        res = b.solve(chunk, tol)
        done_k += chunk
        clock.append((done_k, time.perf_counter() - t0))
        conv = sum(r["status"] == 0 for r in res)
        kk = np.array([r["kkt"] for r in res])
        log(f"iteration {done_k}: {conv}/{len(lps)} converged, max KKT {kk.max():.2e}, "
            f"{clock[-1][1]:.1f}s")
        if conv == len(lps):
            break
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ks = np.array([r["k"] for r in res])
    conv = np.array([r["status"] == 0 for r in res])
    if args.batch_only:
        log(f"batched {t_batch:.1f}s for {done_k} iterations")
        return
    # per-LP single-solve iteration time (3000 iterations incl. 100 checks)
    rates = []
    for i, lp in enumerate(lps):
        s = _lib.Solver(lp, eta=b.info(i)["eta"])
        s.solve(300, 0.0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.solve(3000, 0.0)
        torch.cuda.synchronize()
        rates.append((time.perf_counter() - t1) / 3000)
        s.close()
    rates = np.array(rates)
    t_seq = float(np.sum(ks * rates))
    log(f"batched {t_batch:.1f}s, sequential (sum k_i x rate_i) {t_seq:.1f}s, "
        f"speedup {t_seq / t_batch:.2f}")
    # the converged subset: the batch clock when its last member converged
    sub = None
    if conv.any():
        kc = int(ks[conv].max())
        ck = np.array([c[0] for c in clock])
        ct = np.array([c[1] for c in clock])
        t_sub = float(np.interp(kc, ck, ct))
        t_sub_seq = float(np.sum(ks[conv] * rates[conv]))
        sub = {"lps": int(conv.sum()), "iterations_max": kc,
               "batched_s": round(t_sub, 3), "sequential_plain_s": round(t_sub_seq, 3),
               "speedup": round(t_sub_seq / t_sub, 3),
               "note": "batch clock interpolated inside its chunk of iterations"}
        log(f"converged subset ({conv.sum()} LPs, last at {kc}): batched {t_sub:.1f}s, "
            f"sequential {t_sub_seq:.1f}s")
    # check the sequential model: the three LPs with the fewest iterations
    # solved alone to the tolerance, the three with the most timed alone
    # over a truncated budget (the model uses a rate per iteration)
    checks = []
    order = np.argsort(ks, kind="stable")
    for i in list(order[:3]) + list(order[-3:]):
        i = int(i)
        s = _lib.Solver(lps[i], eta=b.info(i)["eta"])
        few = i in [int(q) for q in order[:3]]
        budget = int(ks[i]) + 30 if few else min(int(ks[i]), args.model_iters)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = s.solve(budget, tol)
        torch.cuda.synchronize()
        checks.append({"lp": i, "kind": "fewest" if few else "most (truncated)",
                       "k": r["k"], "k_batch": int(ks[i]), "converged": r["status"] == 0,
                       "measured_s": round(time.perf_counter() - t1, 3),
                       "model_s": round(float(r["k"] * rates[i]), 3)})
        log(f"model check {checks[-1]}")
        s.close()
    oracle_run = None
    if (~conv).any() and args.oracle_iters > 0:
        oracle_run = unconverged_against_oracle(lps, b, ks, conv, rates, args)
    rerun = None
    if conv.any() and (~conv).any() and not args.no_subset_rerun:
        # the converged subset batched on its own, to the tolerance
        idx = [i for i in range(len(lps)) if conv[i]]
        b2 = _lib.BatchSolver([lps[i] for i in idx],
                              params=[{"eta": b.info(i)["eta"]} for i in idx])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        done2 = 0
        while done2 < args.budget:
            chunk = min(args.chunk, args.budget - done2)
            r2 = b2.solve(chunk, tol)
            done2 += chunk
            c2 = sum(r["status"] == 0 for r in r2)
            log(f"subset iteration {done2}: {c2}/{len(idx)} converged, "
                f"{time.perf_counter() - t1:.1f}s")
            if c2 == len(idx):
                break
        torch.cuda.synchronize()
        t2 = time.perf_counter() - t1
        k2 = np.array([r["k"] for r in r2])
        same = bool(np.array_equal(k2, ks[conv]))
        seq2 = float(np.sum(k2 * rates[conv]))
        rerun = {"lps": len(idx), "all_converged": bool(c2 == len(idx)),
                 "iterations_equal_to_full_batch": same, "batched_s": round(t2, 3),
                 "sequential_plain_s": round(seq2, 3), "speedup": round(seq2 / t2, 3)}
        log(f"converged subset batched alone: {rerun}")
    out = {
        "metric": "time to 1e-8 rel KKT, batched vs plain", "value": round(t_batch, 3),
        "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f64",
        "data": "synthetic", "scaling": "weak", "vs_baseline": None,
        "config": {"workload": f"{len(lps)} planted LPs, m ~ U{{200..20000}}, n = 2m, "
                               f"5 per column, [0,1] (seeds 4000+i)", "tol": tol,
                   "budget": args.budget, "check_period": 30, "restart": "adaptive"},
        "converged": int(conv.sum()), "iterations_max": int(ks.max()),
        "iterations_median": float(np.median(ks)),
        "sequential_plain_s": round(t_seq, 3), "speedup_vs_sequential": round(t_seq / t_batch, 3),
        "converged_subset": sub,
        "converged_subset_batched_alone": rerun,
        "sequential_model_checks": checks,
        "unconverged_member_vs_oracle": oracle_run,
        "single_iteration_us_median": round(float(np.median(rates)) * 1e6, 2),
    }
    print(json.dumps(out), flush=True)


def unconverged_against_oracle(lps, b, ks, conv, rates, args):
    """The unconverged member with the fewest rows: its own GPU solve and
    the oracle (OpenMP build) side by side for the first --oracle-iters
    iterations, check by check: restart decisions, KKT values."""
    import numpy as np
    import oracle
    from paper_2105_12715_amd import _lib
    cand = [i for i in range(len(lps)) if not conv[i]]
    i = min(cand, key=lambda q: lps[q].m)
    lp = lps[i]
    eta = b.info(i)["eta"]
    K = int(args.oracle_iters)
    s = _lib.Solver(lp, eta=eta)
    rg = s.solve(K, args.tol)
    lg = s.check_log(max_records=K // 30 + 1)
    o = oracle.Oracle(lp, eta=eta, mode=oracle.MODE_ADAPTIVE, parallel=True)
    t1 = time.perf_counter()
    ro = o.solve(K, args.tol)
    dt = time.perf_counter() - t1
    lo = o.log()
    n = min(len(lo), len(lg))
    same_int = bool(np.array_equal(lg[:n][:, [0, 1, 2, 9, 10, 11]], lo[:n][:, [0, 1, 2, 9, 10, 11]]))
    kkt_rel = float(np.max(np.abs(lg[:n, 3:5] - lo[:n, 3:5]) / np.maximum(np.abs(lo[:n, 3:5]),
                                                                          1e-300)))
    rep = {"lp": i, "m": lp.m, "n": lp.n, "iterations": K, "checks_compared": n,
           "restart_decisions_equal": same_int, "kkt_max_rel_diff": kkt_rel,
           "gpu_restarts": rg["restarts"], "oracle_restarts": ro["restarts"],
           "gpu_kkt_at_end": rg["kkt"], "oracle_kkt_at_end": ro["kkt"],
           "kkt_every_3000": [float(min(r[3], r[4])) for r in lo[99::100]],
           "oracle_s": round(dt, 2), "oracle_threads": oracle.threads(parallel=True)}
    log(f"unconverged LP {i} against the oracle: {rep}")
    return rep


def run_table2(args):
    """Planted LPs with the sizes of the four Table 2 instances (qap10,
    qap15, nug08-3rd, nug20; the instances themselves are not available):
    the primal-weight search of Section 7 (11 weights 4^-5..4^5, 5000
    iterations without restarts), then the iterations each restart scheme
    needs to bring the KKT error of Table 3 (the largest of the absolute
    primal residual, dual residual and gap) to 1e-6, checked every 30
    iterations with Table 3's limit: no restarts, fixed lengths 4^k (the
    best one reported), adaptive and flexible restarts; for PDHG and the
    extragradient method.  Prints one JSON line with a row per LP and
    method."""
    import torch
    from paper_2105_12715_amd import _lib, lpgen

    names = args.t2_lps.split(",") if args.t2_lps else list(lpgen.TABLE2)
    methods = args.t2_methods.split(",")
    fixed = [int(k) for k in args.t2_fixed.split(",")] if args.t2_fixed else []
    om = [4.0 ** k for k in range(-5, 6)]
    rows = []
    for name in names:
        lp = lpgen.paper_shaped(name)
        for meth in methods:
            mcode = _lib.METHOD_EGM if meth == "egm" else _lib.METHOD_PDHG
            s = _lib.Solver(lp, method=mcode)
            eta = s.info()["eta"]
            t0 = time.perf_counter()
            kk, best, _, _ = s.weight_search(om, 5000)
            torch.cuda.synchronize()
            t_ws = time.perf_counter() - t0
            s.close()
            omega = om[best]
            log(f"{name} {meth}: m={lp.m} n={lp.n} nnz={lp.nnz} eta={eta:.4g}, weight search "
                f"{t_ws:.2f}s -> omega = 4^{best - 5}")
            schemes = [("none", _lib.RESTART_NONE, 0)]
            schemes += [(f"fixed 4^{k}", _lib.RESTART_FIXED, 4 ** k) for k in fixed]
            schemes += [("adaptive", _lib.RESTART_ADAPTIVE, 0),
                        ("flexible", _lib.RESTART_FLEXIBLE, 0)]
            res = {}
            for label, mode, length in schemes:
                s = _lib.Solver(lp, eta=eta, omega=omega, restart_mode=mode, fixed_len=length,
                                kkt_kind=_lib.KKT_MAX_ABS, method=mcode)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = s.solve(args.t2_limit, 1e-6)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                res[label] = {"iterations": r["k"] if r["status"] == 0 else None,
                              "seconds": round(dt, 3), "restarts": r["restarts"]}
                log(f"  {label}: {res[label]}")
                s.close()
            fx = [(v["iterations"], k) for k, v in res.items()
                  if k.startswith("fixed") and v["iterations"] is not None]
            best_fixed = min(fx) if fx else None
            rows.append({"lp": name, "method": meth, "m": lp.m, "n": lp.n, "nnz": lp.nnz,
                         "omega": omega, "weight_search_s": round(t_ws, 3),
                         "no_restarts": res["none"]["iterations"],
                         "best_fixed": best_fixed[0] if best_fixed else None,
                         "best_fixed_length": (4 ** int(best_fixed[1].split("^")[1])
                                               if best_fixed else None),
                         "adaptive": res["adaptive"]["iterations"],
                         "flexible": res["flexible"]["iterations"], "runs": res})
    print(json.dumps({"metric": "iterations to KKT (max abs) <= 1e-6, Table 2 shaped LPs",
                      "unit": "iterations", "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                      "limit": args.t2_limit, "check_period": 30, "rows": rows}), flush=True)


def solver_column_order(lp):
    """The column order the library works in for a single LP (columns by
    entry count, largest first, ties by the row of their first entry):
    returns cinv, the internal index of each of the caller's columns."""
    import numpy as np
    A = lp.scipy_csr().tocsc()
    A.sort_indices()
    cnt = np.diff(A.indptr)
    first = np.full(lp.n, lp.m)
    nz = cnt > 0
    first[nz] = A.indices[A.indptr[:-1][nz]]
    order = np.lexsort((first, -cnt))
    cinv = np.empty(lp.n, np.int64)
    cinv[order] = np.arange(lp.n)
    return cinv


def run_ceiling(args):
    """Ceilings of the GPU for the half-steps, measured with the library's
    own yardstick kernels: a plain streaming copy of 1 GiB (HBM), and plain
    gathers out[i] = val[i] x[idx[i]] with the index streams of the large
    LP's two products (A x+: A's column indices in the solver's column
    order into a 16 MB x; A'y: A''s row indices into an 8 MB y) and with
    uniform random indices into vectors of 4, 8 and 16 MB, each over the
    large LP's entry count; then the gathers alone (pdhg_time_gather_only)
    with the two index streams and with hashed indices over 1 to 16 MB.
    Prints one JSON line."""
    import numpy as np
    import torch
    from paper_2105_12715_amd import _lib, lpgen

    dev = "cuda"
    n = 1 << 27  # 1 GiB of doubles
    src = torch.arange(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    ms = _lib.time_copy(src, dst, reps=20)
    ok = bool(torch.equal(src, dst))
    copy = {"bytes_each_way": 8 * n, "ms": round(ms, 5),
            "gbs_read_plus_write": round(2 * 8 * n / ms / 1e6, 1), "result_checked": ok}
    log(f"copy 1 GiB: {ms:.4f} ms, {copy['gbs_read_plus_write']} GB/s read + write")
    del src, dst
    lp = lpgen.large_powerlaw(3)
    cinv = solver_column_order(lp)
    A = lp.scipy_csr()
    nnz = A.nnz
    At = A.tocsc()
    At.sort_indices()
    rng = np.random.default_rng(7)
    pats = [("A x+ (large LP, x of 16 MB)", cinv[A.indices], lp.n),
            ("A'y (large LP, y of 8 MB)", At.indices[np.argsort(cinv[np.repeat(
                np.arange(lp.n), np.diff(At.indptr))], kind="stable")], lp.m)]
    for mb in (4, 8, 16):
        ln = mb * (1 << 20) // 8
        pats.append((f"uniform over {mb} MB", rng.integers(0, ln, nnz), ln))
    val = torch.as_tensor(np.asarray(A.data), device=dev)
    out = torch.empty(nnz, dtype=torch.float64, device=dev)
    gathers = []
    for name, idx_np, ln in pats:
        idx = torch.as_tensor(np.ascontiguousarray(idx_np, dtype=np.int32), device=dev)
        x = torch.as_tensor(rng.standard_normal(ln), device=dev)
        ms = _lib.time_gather(idx, val, x, out, reps=20)
        ok = bool(torch.equal(out, val * x[idx.long()]))
        rate = nnz / (ms * 1e-3) / 1e9
        gathers.append({"pattern": name, "entries": nnz, "vector_bytes": 8 * ln,
                        "ms": round(ms, 5), "g_gathers_per_s": round(rate, 1),
                        "stream_gbs": round(20 * nnz / ms / 1e6, 1), "result_checked": ok})
        log(f"gather {name}: {ms * 1e3:.1f} us, {rate:.1f} G gathers/s")
    del out
    # the gathers alone (no values, rows or update; 4 per thread, one sum
    # stored per thread): the large LP's two index streams, then hashed
    # indices over windows of 1 to 16 MB (no index stream at all)
    only = []
    for name, idx_np, ln in pats[:2]:
        idx = torch.as_tensor(np.ascontiguousarray(idx_np, dtype=np.int32), device=dev)
        x = torch.as_tensor(rng.standard_normal(ln), device=dev)
        ms, _ = _lib.time_gather_only(x, nnz, idx=idx, reps=20)
        rate = nnz / (ms * 1e-3) / 1e9
        only.append({"pattern": name, "entries": nnz, "vector_bytes": 8 * ln,
                     "ms": round(ms, 5), "g_gathers_per_s": round(rate, 1)})
        log(f"gathers alone, {name}: {ms * 1e3:.1f} us, {rate:.1f} G gathers/s")
    for mb in (1, 2, 4, 8, 16):
        ln = mb * (1 << 20) // 8
        x = torch.as_tensor(rng.standard_normal(ln), device=dev)
        cnt = 1 << 24
        ms, _ = _lib.time_gather_only(x, cnt, reps=20)
        rate = cnt / (ms * 1e-3) / 1e9
        only.append({"pattern": f"hashed indices over {mb} MB", "entries": cnt,
                     "vector_bytes": 8 * ln, "ms": round(ms, 5), "g_gathers_per_s": round(rate, 1)})
        log(f"gathers alone, hashed over {mb} MB: {ms * 1e3:.1f} us, {rate:.1f} G gathers/s")
    print(json.dumps({"metric": "yardstick ceilings", "dtype": "f64", "n_gpus": 1,
                      "copy": copy, "gather": gathers, "gathers_alone": only}), flush=True)


def run_to_tol(args, lp, wdesc):
    """Time to relative KKT <= tol from the initial point (pdhg_solve with
    checks every 30 iterations), with the oracle's time for the same
    iteration count projected from a bounded sample of its iterations."""
    import torch
    from paper_2105_12715_amd import _lib
    s = _lib.Solver(lp, restart_mode=_lib.RESTART_ADAPTIVE)
    torch.cuda.synchronize()
    eta = s.info()["eta"]
    t0 = time.perf_counter()
    r = s.solve(args.budget, args.tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"{wdesc}: status {r['status']} after {r['k']} iterations, {r['restarts']} restarts, "
        f"KKT {r['kkt']:.3e}, {dt:.3f}s")
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle solved to the same tolerance (measured, not projected):
        # the OpenMP build on every host core and the plain build on one
        import oracle
        runs = {}
        for par in (True, False):
            o = oracle.Oracle(lp, eta=eta, mode=oracle.MODE_ADAPTIVE, parallel=par)
            t0 = time.perf_counter()
            ro = o.solve(args.budget, args.tol)
            runs[par] = (time.perf_counter() - t0, ro)
            o.close()
            log(f"oracle ({'all cores' if par else 'one core'}): status {ro['status']} after "
                f"{ro['k']} iterations, {ro['restarts']} restarts, {runs[par][0]:.2f}s")
        (dp, rp_), (d1, r1) = runs[True], runs[False]
        cpu = {"value": round(dp, 3), "unit": "s", "cores": oracle.threads(parallel=True),
               "kind": "oracle",
               "sample": f"the whole solve to {args.tol:g}: {rp_['k']} iterations, "
                         f"{rp_['restarts']} restarts, OpenMP build (bitwise the plain "
                         f"build's iterates)",
               "one_core": {"value": round(d1, 3), "unit": "s", "cores": 1,
                            "iterations": r1["k"], "restarts": r1["restarts"]}}
    out = {"metric": f"time to {args.tol:g} rel KKT", "value": round(dt, 4), "unit": "s",
           "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "scaling": "weak", "vs_baseline": None,
           "config": {"workload": wdesc, "m": lp.m, "n": lp.n, "nnz": lp.nnz, "tol": args.tol,
                      "check_period": 30, "restart": "adaptive"},
           "converged": r["status"] == 0, "iterations": r["k"], "restarts": r["restarts"],
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def run_adjoint(args):
    """Differentiation workload: 32 planted LPs of 5000 x 10000 (5 per
    column), K = 2000 unrolled iterations, loss |x_K - x_target|^2; times of
    the forward pass (with its checkpoints) and of the reverse pass, and the
    oracle's forward + reverse time for one member, times 32."""
    import numpy as np
    import torch
    from paper_2105_12715_amd import _lib, lpgen
    K = args.adj_k
    lps = [lpgen.diff_member(i) for i in range(32)]
    b = _lib.BatchSolver(lps)
    xt = torch.as_tensor(np.concatenate([lpgen.x_target(i, lp.n) for i, lp in enumerate(lps)]),
                         device="cuda:0")
    b.unrolled_forward(60)  # warm-up of the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xk, tape = b.unrolled_forward(K)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    gc, gb, gA = b.unrolled_backward(tape, 2.0 * (xk - xt))
    torch.cuda.synchronize()
    t_rev = time.perf_counter() - t0
    log(f"forward {t_fwd:.3f}s, reverse {t_rev:.3f}s for 32 LPs, K = {K}")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.Oracle(lps[0], eta=b.info(0)["eta"])
        t0 = time.perf_counter()
        o.unrolled_grad(K, lpgen.x_target(0, lps[0].n))
        one = time.perf_counter() - t0
        cpu = {"value": round(32 * one, 2), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": f"forward + reverse of member 0 on one core ({one:.1f} s), times 32"}
    out = {"metric": "time of K unrolled iterations and their reverse pass", "value":
           round(t_fwd + t_rev, 4), "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f64", "data": "synthetic", "scaling": "weak", "vs_baseline": None,
           "config": {"workload": "32 planted LPs 5000 x 10000, 5 per column, [0,1] "
                                  "(seeds 5000+i)", "K": K, "loss": "|x_K - x_target|^2"},
           "forward_s": round(t_fwd, 4), "reverse_s": round(t_rev, 4), "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def run_many(args):
    """Many small LPs to --tol: each 50 x 100 LP (seeds 1..N) solved alone
    one after another, all of them in one pdhg_solve_many call (one
    workgroup per LP), and all of them through the batched solver
    (pdhg_batch_*); plus the oracle on a few of them, projected to N."""
    import numpy as np
    import torch
    from paper_2105_12715_amd import _lib, lpgen
    N = args.many_count
    lps = [lpgen.small_dense(1 + i) for i in range(N)]
    wdesc = f"{N} small LPs 50 x 100, Bernoulli(0.1) (seeds 1..{N})"
    log(f"workload {wdesc}")

    def fresh():
        return [_lib.Solver(lp) for lp in lps]

    seq = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r_seq = [s.solve(args.budget, args.tol) for s in seq]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    log(f"one after another: {t_seq:.3f} s")
    many = fresh()
    assert all(s.info()["one_workgroup"] for s in many)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r_many = _lib.solve_many(many, args.budget, args.tol)
    torch.cuda.synchronize()
    t_many = time.perf_counter() - t0
    log(f"pdhg_solve_many: {t_many:.3f} s")
    if r_many != r_seq:
        raise SystemExit("pdhg_solve_many differs from the single solves")
    b = _lib.BatchSolver(lps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r_b = b.solve(args.budget, args.tol)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batched solver: {t_batch:.3f} s")
    ks = [r["k"] for r in r_seq]
    nconv = sum(r["status"] == 0 for r in r_seq)
    line = {"metric": f"time to {args.tol:g} rel KKT", "value": round(t_many, 4), "unit": "s",
            "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
            "scaling": "weak", "vs_baseline": None,
            "config": {"workload": wdesc, "count": N, "tol": args.tol, "budget": args.budget,
                       "check_period": 30, "restart": "adaptive"},
            "converged": nconv, "iterations_total": int(sum(ks)),
            "iterations_median": int(np.median(ks)), "iterations_max": int(max(ks)),
            "one_after_another_s": round(t_seq, 4), "batched_solver_s": round(t_batch, 4),
            "batched_solver_converged": int(sum(r["status"] == 0 for r in r_b)),
            "speedup_vs_one_after_another": round(t_seq / t_many, 2),
            "lp_iterations_per_s": round(sum(ks) / t_many, 1)}
    if not args.no_cpu_baseline:
        import oracle
        sample = lps[: min(8, N)]
        t0 = time.perf_counter()
        for lp in sample:
            oracle.Oracle(lp, eta=_lib.Solver(lp).info()["eta"]).solve(args.budget, args.tol)
        t_cpu = (time.perf_counter() - t0) / len(sample) * N
        line["cpu_baseline"] = {"value": round(t_cpu, 3), "unit": "s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"{len(sample)} of the LPs solved to {args.tol:g} by "
                                          "the single-threaded FP64 C oracle, scaled to "
                                          f"{N} LPs"}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed blocks of 30 iterations (default 167; 2000 for the small LP, "
                         "whose blocks take microseconds)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="large",
                    choices=["large", "medium", "small", "batch", "table2", "adjoint", "many",
                             "ceiling"])
    ap.add_argument("--many-count", type=int, default=256)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-only", action="store_true",
                    help="batch: skip the sequential single-LP timings (for profiling)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--budget", type=int, default=1_500_000)
    ap.add_argument("--chunk", type=int, default=30_000)
    ap.add_argument("--model-iters", type=int, default=30_000,
                    help="batch: truncated budget of the model check on the slowest LPs")
    ap.add_argument("--no-subset-rerun", action="store_true",
                    help="batch: skip the rerun of the converged subset as a batch of its own")
    ap.add_argument("--oracle-iters", type=int, default=30_000,
                    help="batch: iterations of the unconverged member run by the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="large/medium/small: time the SpMV schedule on the LP first "
                         "(pdhg_autotune) instead of the default")
    ap.add_argument("--kernel-iters", type=int, default=200)
    ap.add_argument("--to-tol", action="store_true",
                    help="large/medium/small: time to --tol instead of iterations per second")
    ap.add_argument("--adj-k", type=int, default=2000)
    ap.add_argument("--t2-lps", default="", help="table2: comma list of Table 2 names")
    ap.add_argument("--t2-methods", default="pdhg,egm")
    ap.add_argument("--t2-fixed", default="1,2,3,4,5,6,7,8,9", help="table2: exponents k of 4^k")
    ap.add_argument("--t2-limit", type=int, default=500_000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the library's plain 1 GiB copy kernel five times, the "
                         "yardstick for the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2105_12715_amd import _lib

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    _lib.load(build_if_missing=True)
    if args.calibrate_copy:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        _lib.time_copy(x, y, reps=4)  # warm-up launch + 4 timed: 5 launches
        torch.cuda.synchronize()
        log("copy calibration: 5 launches of the library's copy kernel, 1073741824 bytes "
            "read and written each")
        return
    if args.workload == "ceiling":
        run_ceiling(args)
        return
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "table2":
        run_table2(args)
        return
    if args.workload == "adjoint":
        run_adjoint(args)
        return
    if args.workload == "many":
        run_many(args)
        return
    t0 = time.perf_counter()
    lp, wdesc = make_workload(args.workload)
    log(f"workload {wdesc}: m={lp.m} n={lp.n} nnz={lp.nnz} generated in "
        f"{time.perf_counter() - t0:.1f}s")
    if args.to_tol:
        run_to_tol(args, lp, wdesc)
        return
    t0 = time.perf_counter()
    s = _lib.Solver(lp, restart_mode=_lib.RESTART_ADAPTIVE)
    torch.cuda.synchronize()
    info = s.info()
    log(f"setup (validate, transpose, power iteration {info['power_iters_used']} steps) "
        f"{time.perf_counter() - t0:.2f}s, eta={info['eta']:.6g}")
    tune = None
    if args.autotune:
        # the per-matrix SpMV schedule (column slabs, then lanes per row),
        # timed on this LP before the timed region.  Off by default: on the
        # large LP the tuner keeps the default slabs and moves the lanes of
        # A x by one step for well under 1 us, and under a profiler (which
        # serializes kernels) it can pick another schedule than in the timed
        # run, so the profiles and the line keep the default schedule.
        t0 = time.perf_counter()
        tune = s.autotune(iters=10, use_cache=False)
        log(f"autotune {time.perf_counter() - t0:.2f}s: {tune}")
    P = 30
    if args.steps is None:
        args.steps = 2000 if args.workload == "small" else 167
    s.solve(args.warmup * P, 0.0)
    torch.cuda.synchronize()
    log("warmup done")
    t0 = time.perf_counter()
    s.solve(args.steps * P, 0.0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = args.steps * P
    value = iters / dt
    info = s.info()
    log(f"timed {iters} iterations in {dt:.3f}s: {value:.1f} iter/s, restarts so far "
        f"{info['restarts']}")

    ms_p, ms_d = s.time_iterations(args.kernel_iters)
    m, n, nnz = lp.m, lp.n, lp.nnz
    bytes_p, bytes_d = halfstep_bytes(m, n, nnz)
    if ms_p >= ms_d:
        kname, kb, kms = "primal", bytes_p, ms_p
    else:
        kname, kb, kms = "dual", bytes_d, ms_d
    achieved = kb / (kms * 1e-3) / 1e9
    log(f"kernel ms: primal {ms_p:.4f} ({bytes_p / ms_p / 1e6:.0f} GB/s), dual {ms_d:.4f} "
        f"({bytes_d / ms_d / 1e6:.0f} GB/s)")
    traffic = measured_traffic(args.workload, kname)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"{kname} half-step SpMV", "algorithmic_bytes_per_launch": kb,
            "ms_per_launch": round(kms, 5),
            "other_kernel_ms": round(ms_d if kname == "primal" else ms_p, 5)}
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(lp, info["eta"])
        log(f"cpu baseline {cpu['value']:.2f} iter/s")
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wdesc, "m": m, "n": n, "nnz": nnz, "check_period": P,
                   "iterations_per_step": P, "restart": "adaptive", "parallelism": "single GPU",
                   "schedule": None if tune is None else {
                       k: tune[k] for k in ("slabs_A", "slabs_At", "lanes_bias_A",
                                            "lanes_bias_At")}},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    s.close()


if __name__ == "__main__":
    main()
