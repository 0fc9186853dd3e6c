"""The rocprofv3 summary helper behind the committed profiles: kernel-trace
statistics and the HBM traffic of a half-step from FETCH_SIZE / WRITE_SIZE
runs scaled by a copy kernel of known size (synthetic CSV files, no GPU)."""
import argparse
import csv
import os

from paper_2105_12715_amd import profsum


def _counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_traffic_scales_by_the_copy_kernel(tmp_path):
    gib = 1 << 30
    # the copy reads and writes 1 GiB; its counters read half and all of it
    _counters(tmp_path / "cf", [(1, "neg_kernel(double*)", "FETCH_SIZE", gib / 2 / 1024)])
    _counters(tmp_path / "cw", [(1, "neg_kernel(double*)", "WRITE_SIZE", gib / 1024)])
    # two dispatches of each half-step kernel, per-XCD rows summed per dispatch
    _counters(tmp_path / "f", [
        (10, "void pdhg::k_a<X>(int)", "FETCH_SIZE", 100.0), (10, "void pdhg::k_a<X>(int)", "FETCH_SIZE", 50.0),
        (11, "void pdhg::k_a<X>(int)", "FETCH_SIZE", 130.0), (11, "void pdhg::k_a<X>(int)", "FETCH_SIZE", 20.0),
        (12, "void pdhg::k_b<Y>(int)", "FETCH_SIZE", 40.0)])
    _counters(tmp_path / "w", [
        (10, "void pdhg::k_a<X>(int)", "WRITE_SIZE", 8.0), (11, "void pdhg::k_a<X>(int)", "WRITE_SIZE", 12.0),
        (12, "void pdhg::k_b<Y>(int)", "WRITE_SIZE", 6.0)])
    a = argparse.Namespace(fetch=str(tmp_path / "f"), write=str(tmp_path / "w"),
                           copy_fetch=str(tmp_path / "cf"), copy_write=str(tmp_path / "cw"),
                           copy_bytes=gib, copy_kernel="neg_kernel", kernels="k_a<X>,k_b<Y>",
                           source_hash="abc", cmd="cmd")
    r = profsum.traffic(a)
    assert r["fetch_scale"] == 2.0 and r["write_scale"] == 1.0
    ka = r["kernels"]["pdhg::k_a<X>"]
    kb = r["kernels"]["pdhg::k_b<Y>"]
    # k_a: 150 KiB per dispatch fetched (x 2), 10 KiB written (x 1)
    assert ka == {"fetch_bytes": 150 * 1024 * 2, "write_bytes": 10 * 1024, "dispatches": 1}
    assert kb == {"fetch_bytes": 40 * 1024 * 2, "write_bytes": 6 * 1024, "dispatches": 1}
    assert r["hbm_bytes_per_launch"] == (300 + 10 + 80 + 6) * 1024
    assert r["kernel_source_hash"] == "abc"
    # k_a dispatched twice per half-step (two column slabs of one product)
    a.kernels = "k_a<X>*2,k_b<Y>"
    r2 = profsum.traffic(a)
    assert r2["kernels"]["pdhg::k_a<X>"] == {"fetch_bytes": 150 * 1024 * 2 * 2,
                                             "write_bytes": 10 * 1024 * 2, "dispatches": 2}
    assert r2["hbm_bytes_per_launch"] == (600 + 20 + 80 + 6) * 1024


def test_stats_table(tmp_path):
    d = tmp_path / "s"
    os.makedirs(d)
    with open(d / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writerow(["void pdhg::k_small(int)", 4, 4000, 1000, 20.0])
        w.writerow(["void pdhg::k_big(int)", 2, 16000, 8000, 80.0])
    md = profsum.stats_markdown(str(d), "T", "C")
    lines = [l for l in md.splitlines() if l.startswith("| `")]
    assert lines[0] == "| `pdhg::k_big` | 2 | 16.0 | 8.000 | 80.00 |"
    assert lines[1] == "| `pdhg::k_small` | 4 | 4.0 | 1.000 | 20.00 |"
