"""Summaries of rocprofv3 output for the benchmark's roofline record.

    python rocprof_summary.py trace  <kernel_stats.csv>
    python rocprof_summary.py traffic <fetch_counter.csv> <write_counter.csv> \
        --out profiles/c1_fused_steps_traffic.json --workload c1
    python rocprof_summary.py l2 <tcc_counter.csv>

`trace` prints a per-kernel table (calls, mean/min/max duration); `l2`
prints mean L2 (TCC) requests, hits, misses and the hit rate per dispatch of
each kernel (requests only when the run collected TCC_REQ_sum).  `traffic`
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
    m = re.search(r"(k_\w+)<dpdlp::(\w+)(?:<\s*(\w+)\s*>)?", name)
    if m:
        inner = m.group(2) + (f"<{m.group(3)}>" if m.group(3) else "")
        return f"{m.group(1)}<{inner}>"
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
    """[(dispatch id, kernel name, value)] in dispatch order (values of one
    dispatch summed over the counter's instances)."""
    with open(path) as f:
        rows = list(csv.reader(f))
    h = rows[0]
    i_n = _col(h, "kernel_name")
    i_cn = _col(h, "counter_name")
    i_cv = _col(h, "counter_value")
    i_d = _col(h, "dispatch_id")
    per = {}
    for r in rows[1:]:
        if r[i_cn] != counter:
            continue
        d = int(r[i_d])
        name, v = per.get(d, (r[i_n], 0.0))
        per[d] = (name, v + float(r[i_cv]))
    return [(d, per[d][0], per[d][1]) for d in sorted(per)]


def step_of(name):
    """Which fused step a kernel belongs to: ('primal' | 'dual', is_head),
    'partial' for the per-slice partial sums (the step is named by the
    combine that follows), or None.  FP64 and FP32 steps alike (a run
    profiles one precision)."""
    for op, step in (("PrimalOp<", "primal"), ("DualOp<", "dual")):
        if op in name:
            head = "k_tile<" in name or "k_combine<" in name
            return step, head
    if "PartialOp<double>" in name or "PartialOp<float>" in name:
        return "partial"
    return None


def per_step_bytes(disp):
    """Mean counter value (KiB for FETCH_SIZE / WRITE_SIZE) per launch of each
    fused step.  A step is the tile
    kernel and its split-segment fix-up or, in the XCD-sliced form, the
    per-slice partial kernel (and fix-up) and the combine kernel that follows
    it; partial kernels followed by another pass's combine are dropped."""
    tot, launches, pending = defaultdict(float), defaultdict(int), 0.0
    for _, name, v in disp:
        s = step_of(name)
        if s is None:
            if "k_combine<" in name:      # partial sums of another pass (checks, SpMV, Lanczos)
                pending = 0.0
            continue
        if s == "partial":
            pending += v
            continue
        step, head = s
        tot[step] += v
        if "k_combine<" in name:
            tot[step] += pending
            pending = 0.0
        if head:
            launches[step] += 1
    return {k: (tot[k] / launches[k], launches[k]) for k in launches}


def kernel_source_hash(root):
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(root, "paper_2601_07628_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic(fetch_csv, write_csv, workload, tcc_csv=None):
    fe = read_counter(fetch_csv, "FETCH_SIZE")
    wr = read_counter(write_csv, "WRITE_SIZE")

    def first_copy(disp):
        for _, name, v in disp:
            if "copy" in name.lower():
                return name, v
        raise SystemExit("no calibration copy kernel found in the counter run")
    # the first copy dispatch is the 256 MiB calibration copy
    cname, cf = first_copy(fe)
    _, cw = first_copy(wr)
    cal_f, cal_w = CALIB_BYTES / (cf * 1024.0), CALIB_BYTES / (cw * 1024.0)
    out = {"calibration": {"copy_kernel": short_name(cname),
                           "fetch_factor": cal_f, "write_factor": cal_w}, "kernels": {}}
    sf, sw = per_step_bytes(fe), per_step_bytes(wr)
    for step, (f_kib, n) in sf.items():
        w_kib = sw.get(step, (0.0, 0))[0]
        f_b, w_b = f_kib * 1024.0 * cal_f, w_kib * 1024.0 * cal_w
        out["kernels"][f"{workload}/{step}"] = {
            "launches": n, "fetch_bytes_per_launch": f_b,
            "write_bytes_per_launch": w_b, "bytes_per_launch": f_b + w_b}
    if tcc_csv:
        # L2 requests of each fused step (its partial-sum and combine
        # kernels together), from a TCC_REQ_sum / TCC_HIT_sum run
        for ctr, key in (("TCC_REQ_sum", "l2_requests_per_launch"),
                         ("TCC_HIT_sum", "l2_hits_per_launch")):
            for step, (v, n) in per_step_bytes(read_counter(tcc_csv, ctr)).items():
                out["kernels"].setdefault(f"{workload}/{step}", {})[key] = v
    per_kernel = defaultdict(list)
    for _, name, v in fe:
        per_kernel[short_name(name)].append(v)
    out["fetch_kib_per_dispatch"] = {k: round(sum(v) / len(v), 1) for k, v in per_kernel.items()}
    per_kernel = defaultdict(list)
    for _, name, v in wr:
        per_kernel[short_name(name)].append(v)
    out["write_kib_per_dispatch"] = {k: round(sum(v) / len(v), 1) for k, v in per_kernel.items()}
    return out


def l2_table(path):
    hits = read_counter(path, "TCC_HIT_sum")
    miss = {d: v for d, _, v in read_counter(path, "TCC_MISS_sum")}
    req = {d: v for d, _, v in read_counter(path, "TCC_REQ_sum")}
    per = defaultdict(lambda: [0, 0.0, 0.0, 0.0])
    for d, name, h in hits:
        e = per[short_name(name)]
        e[0] += 1
        e[1] += h
        e[2] += miss.get(d, 0.0)
        e[3] += req.get(d, 0.0)
    rows = []
    for k, (n, h, m, q) in per.items():
        rows.append((k, n, q / n, h / n, m / n, h / (h + m) if h + m > 0 else 0.0))
    rows.sort(key=lambda r: -(r[3] + r[4]) * r[1])
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats_csv")
    l2 = sub.add_parser("l2")
    l2.add_argument("counter_csv")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("--out", required=True)
    c.add_argument("--workload", default="c1")
    c.add_argument("--tcc", default=None, help="TCC_REQ_sum / TCC_HIT_sum counter run")
    c.add_argument("--command", default="")
    a = ap.parse_args(argv)
    if a.cmd == "l2":
        print(f"{'kernel':44s} {'calls':>6s} {'req/disp':>12s} {'hits/disp':>12s} "
              f"{'misses/disp':>12s} {'hit rate':>9s}")
        for k, n, q, h, m, r in l2_table(a.counter_csv):
            print(f"{k:44s} {n:6d} {q:12.0f} {h:12.0f} {m:12.0f} {r:9.3f}")
    elif a.cmd == "trace":
        rows = read_trace(a.stats_csv)
        print(f"{'kernel':44s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s}")
        for r in rows:
            print(f"{r['short']:44s} {r['calls']:6d} {r['total_ms']:10.3f} {r['avg_us']:9.2f} "
                  f"{r['min_us']:9.2f} {r['max_us']:9.2f}")
    else:
        root = os.path.dirname(os.path.abspath(__file__))
        d = traffic(a.fetch_csv, a.write_csv, a.workload, a.tcc)
        d["source_hash"] = kernel_source_hash(root)
        d["command"] = a.command
        with open(a.out, "w") as f:
            json.dump(d, f, indent=1)
        json.dump(d, sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()
