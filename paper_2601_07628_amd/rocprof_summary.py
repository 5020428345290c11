"""Summaries of rocprofv3 output for the benchmark's roofline record.

    python -m paper_2601_07628_amd.rocprof_summary trace  <kernel_stats.csv>
    python -m paper_2601_07628_amd.rocprof_summary traffic <fetch_counter.csv> <write_counter.csv> \
        --out profiles/traffic.json --workload c1

`trace` prints a per-kernel table (calls, mean/min/max duration).  `traffic`
turns two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs (KiB per dispatch)
into HBM bytes per launch of the fused kernels.  The counters are calibrated
by the 256 MiB device-to-device copy that ``bench.py --calib-copy`` runs first
(268435456 bytes read and written): factor = known bytes / counted bytes.
The output records the hash of the kernel sources it was taken on; bench.py
reports the traffic only while that hash matches.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import re
import sys
from collections import defaultdict

CALIB_BYTES = 268435456


def _col(header, *names):
    low = [h.lower() for h in header]
    for n in names:
        if n in low:
            return low.index(n)
    raise KeyError(f"none of {names} in {header}")


def short_name(name: str) -> str:
    m = re.search(r"k_tile<dpdlp::(\w+)(?:<(\w+)>)?", name)
    if m:
        return f"k_tile<{m.group(1)}{'<' + m.group(2) + '>' if m.group(2) else ''}>"
    m = re.search(r"(k_\w+)", name)
    if m:
        return m.group(1)
    return name[:60]


def read_trace(path):
    with open(path) as f:
        rows = list(csv.reader(f))
    h = rows[0]
    i_n, i_c = _col(h, "name", "kernel_name"), _col(h, "calls")
    i_t, i_a = _col(h, "totaldurationns"), _col(h, "averagens")
    i_mn, i_mx = _col(h, "minns"), _col(h, "maxns")
    out = []
    for r in rows[1:]:
        out.append(dict(name=r[i_n], short=short_name(r[i_n]), calls=int(r[i_c]),
                        total_ms=float(r[i_t]) / 1e6, avg_us=float(r[i_a]) / 1e3,
                        min_us=float(r[i_mn]) / 1e3, max_us=float(r[i_mx]) / 1e3))
    return out


def read_counter(path, counter):
    """{kernel name: [values per dispatch, in dispatch order]}"""
    with open(path) as f:
        rows = list(csv.reader(f))
    h = rows[0]
    i_n = _col(h, "kernel_name")
    i_cn = _col(h, "counter_name")
    i_cv = _col(h, "counter_value")
    i_d = _col(h, "dispatch_id")
    per = defaultdict(dict)
    for r in rows[1:]:
        if r[i_cn] != counter:
            continue
        per[r[i_n]][int(r[i_d])] = per[r[i_n]].get(int(r[i_d]), 0.0) + float(r[i_cv])
    return {k: [v[d] for d in sorted(v)] for k, v in per.items()}


def kernel_source_hash(root):
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(root, "paper_2601_07628_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic(fetch_csv, write_csv, workload):
    fe = read_counter(fetch_csv, "FETCH_SIZE")
    wr = read_counter(write_csv, "WRITE_SIZE")
    copy = [k for k in fe if "copy" in k.lower()]
    if not copy:
        raise SystemExit("no calibration copy kernel found in the FETCH_SIZE run")
    # the first copy dispatch is the 256 MiB calibration copy
    cal_f = CALIB_BYTES / (fe[copy[0]][0] * 1024.0)
    wc = [k for k in wr if "copy" in k.lower()]
    cal_w = CALIB_BYTES / (wr[wc[0]][0] * 1024.0)
    out = {"calibration": {"copy_kernel": short_name(copy[0]),
                           "fetch_factor": cal_f, "write_factor": cal_w}, "kernels": {}}
    for name, vals in fe.items():
        key = None
        if "PrimalOp<double>" in name:
            key = "primal"
        elif "DualOp<double>" in name:
            key = "dual"
        if key is None:
            continue
        wv = wr.get(name, [])
        f_b = sum(vals) / len(vals) * 1024.0 * cal_f
        w_b = (sum(wv) / len(wv) * 1024.0 * cal_w) if wv else 0.0
        out["kernels"][f"{workload}/{key}"] = {
            "dispatches": len(vals), "fetch_bytes_per_launch": f_b,
            "write_bytes_per_launch": w_b, "bytes_per_launch": f_b + w_b,
            "kernel": short_name(name)}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats_csv")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("--out", required=True)
    c.add_argument("--workload", default="c1")
    c.add_argument("--command", default="")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        rows = read_trace(a.stats_csv)
        print(f"{'kernel':44s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s}")
        for r in rows:
            print(f"{r['short']:44s} {r['calls']:6d} {r['total_ms']:10.3f} {r['avg_us']:9.2f} "
                  f"{r['min_us']:9.2f} {r['max_us']:9.2f}")
    else:
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        d = traffic(a.fetch_csv, a.write_csv, a.workload)
        d["source_hash"] = kernel_source_hash(root)
        d["command"] = a.command
        with open(a.out, "w") as f:
            json.dump(d, f, indent=1)
        json.dump(d, sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()
