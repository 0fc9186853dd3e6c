"""Summaries of rocprofv3 CSV output for the kernels of this library.

    python -m paper_2105_12715_amd.profsum stats DIR --title T --cmd C
        markdown table of the kernel-trace statistics found under DIR
    python -m paper_2105_12715_amd.profsum pmc DIR [DIR ...]
        mean of every collected counter per dispatch, per kernel
    python -m paper_2105_12715_amd.profsum traffic --fetch D1 --write D2
            --copy-fetch D3 --copy-write D4 --copy-bytes B --kernels K1,K2*2
            --source-hash H --cmd C
        HBM bytes per launch of the kernels K1 + K2 (one half-step) from
        FETCH_SIZE and WRITE_SIZE runs, each scaled by what the same counter
        reads for a copy kernel that moves B bytes each way (JSON); K*n
        counts n dispatches of kernel K per half-step (the column slabs of
        one product run the same kernel once per slab)

Runs on the host on files that rocprofv3 wrote (``--output-format csv``);
nothing here touches a GPU.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys
from collections import defaultdict


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits


def _col(row, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n in low:
            return row[low[n]]
    raise KeyError(f"none of {names} in {list(row)}")


def short_name(n):
    n = n.split("(")[0].replace("void ", "").strip()
    return n


def kernel_stats(d):
    rows = []
    for f in _find(d, "kernel_stats.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((short_name(_col(r, "name")), int(_col(r, "calls")),
                             float(_col(r, "totaldurationns")) / 1e3,
                             float(_col(r, "averagens")) / 1e3,
                             float(_col(r, "percentage"))))
    rows.sort(key=lambda t: -t[2])
    return rows


def stats_markdown(d, title, cmd, top=30):
    out = [f"# {title}", "", "Command (from the repository root, TMPDIR=/tmp):", "", "```", cmd,
           "```", "", "rocprofv3 kernel-trace statistics (microseconds):", "",
           "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for n, c, t, a, p in kernel_stats(d)[:top]:
        out.append(f"| `{n}` | {c} | {t:.1f} | {a:.3f} | {p:.2f} |")
    return "\n".join(out) + "\n"


def counters_per_dispatch(dirs):
    """{kernel: {counter: mean value per dispatch}} and dispatch counts."""
    acc = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        for f in _find(d, "counter_collection.csv"):
            with open(f) as fh:
                per = defaultdict(float)
                names = {}
                for r in csv.DictReader(fh):
                    key = (_col(r, "dispatch_id"), _col(r, "counter_name"))
                    per[key] += float(_col(r, "counter_value"))
                    names[key[0]] = short_name(_col(r, "kernel_name"))
                for (disp, cn), v in per.items():
                    acc[names[disp]][cn].append(v)
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}, \
        {k: max(len(v) for v in cs.values()) for k, cs in acc.items()}


def _match(stats, pattern):
    hits = [k for k in stats if pattern in k]
    if len(hits) != 1:
        raise SystemExit(f"kernel pattern {pattern!r} matches {hits}")
    return hits[0]


def traffic(a):
    fetch, _ = counters_per_dispatch([a.fetch])
    write, _ = counters_per_dispatch([a.write])
    cfetch, _ = counters_per_dispatch([a.copy_fetch])
    cwrite, _ = counters_per_dispatch([a.copy_write])
    ck = _match(cfetch, a.copy_kernel)
    kib = 1024.0
    f_scale = a.copy_bytes / (cfetch[ck]["FETCH_SIZE"] * kib)
    w_scale = a.copy_bytes / (cwrite[_match(cwrite, a.copy_kernel)]["WRITE_SIZE"] * kib)
    parts = {}
    total = 0.0
    for item in a.kernels.split(","):
        pat, _, times = item.partition("*")
        n = int(times) if times else 1
        kf, kw = _match(fetch, pat), _match(write, pat)
        fb = fetch[kf]["FETCH_SIZE"] * kib * f_scale * n
        wb = write[kw]["WRITE_SIZE"] * kib * w_scale * n
        parts[kf] = {"fetch_bytes": round(fb), "write_bytes": round(wb), "dispatches": n}
        total += fb + wb
    return {"kernels": parts, "hbm_bytes_per_launch": round(total),
            "counts": "bytes between L2 and the memory fabric (FETCH_SIZE, WRITE_SIZE), "
                      "scaled by the copy yardstick; reads served by the MALL (Infinity "
                      "Cache) count too, so this is an upper bound on DRAM bytes",
            "copy_kernel": ck, "copy_bytes_each_way": a.copy_bytes,
            "fetch_scale": f_scale, "write_scale": w_scale,
            "kernel_source_hash": a.source_hash, "command": a.cmd}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--title", required=True)
    s.add_argument("--cmd", required=True)
    p = sub.add_parser("pmc")
    p.add_argument("dirs", nargs="+")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "kernels", "source_hash", "cmd"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--copy-kernel", default="k_copy_yard")
    a = ap.parse_args(argv)
    if a.what == "stats":
        sys.stdout.write(stats_markdown(a.dir, a.title, a.cmd))
    elif a.what == "pmc":
        vals, cnt = counters_per_dispatch(a.dirs)
        for k in sorted(vals):
            print(k, cnt[k], json.dumps({c: round(v, 1) for c, v in vals[k].items()}))
    else:
        print(json.dumps(traffic(a), indent=1))


if __name__ == "__main__":
    main()
