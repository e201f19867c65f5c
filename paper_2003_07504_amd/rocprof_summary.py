"""Summarise rocprofv3 output (rocpd SQLite databases) of a bench.py run.

    python -m paper_2003_07504_amd.rocprof_summary --trace KT.db --fetch F.db \
        --write W.db [--sq S.db] --size 1080x1920x3 --command "<rocprofv3 ...>" \
        --out profiles/ils_passes_1080p_rgb_n4.txt

Writes a short text summary (per-kernel call counts and durations, HBM bytes
per launch from FETCH_SIZE / WRITE_SIZE scaled by what the same counters
read for a 512 MiB device copy, SQ counters) and records the bytes per
launch in profiles/traffic.json under the current kernel-source hash, which
bench.py uses for the roofline's `traffic` field.
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import re
import sqlite3

from .build import source_hash

COPY_BYTES = 1 << 29
KINDS = {"0": "row_first", "1": "row_mid", "2": "row_final", "3": "row_first"}


def kind_of(name: str) -> str:
    m = re.search(r"k_row<(\d+), (\d+), (\d+), (\d), (\d)>", name)
    if m:
        return KINDS[m.group(4)] + ("_welsch" if m.group(5) == "1" else "")
    if re.search(r"k_col<", name):
        return "column"
    if "copyBuffer" in name:
        return "copy"
    return re.sub(r"\(.*", "", name)[:48]


def trace(db):
    """Per pass kind, the kernel instance launched most often (the tuner also
    times the other tile shapes a few times) with its duration statistics."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), avg(duration), min(duration), max(duration) "
                       "from kernels group by name").fetchall()
    out = {}
    for n, c, a, lo, hi in rows:
        k = kind_of(n)
        if k not in out or c > out[k][1]:
            out[k] = (n, c, a / 1e3, lo / 1e3, hi / 1e3)
    return out


def timeline(db, chosen, npass):
    """Whole steps in the trace: runs of the chosen pass kernels from a first
    row pass to a final row pass, npass launches long.  Returns the medians
    of (span from the first start to the last end, sum of kernel durations,
    sum of the gaps between consecutive launches) in microseconds, and the
    number of steps found."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    names = {v[0]: k for k, v in chosen.items()}
    steps, cur = [], []
    for n, st, en in rows:
        k = names.get(n)
        if k is None:
            continue
        if k == "row_first":
            cur = [(st, en)]
        elif cur:
            cur.append((st, en))
            if k == "row_final":
                if len(cur) == npass:
                    steps.append(cur)
                cur = []
    if not steps:
        return None
    def med(v):
        v = sorted(v)
        return v[len(v) // 2] / 1e3
    span = med([s[-1][1] - s[0][0] for s in steps])
    busy = med([sum(e - b for b, e in s) for s in steps])
    gaps = med([sum(max(0, s[i + 1][0] - s[i][1]) for i in range(len(s) - 1)) for s in steps])
    return span, busy, gaps, len(steps)


def counters(db, largest=False):
    """{kernel name: {counter: average value per dispatch}}, or the largest
    value of any dispatch when largest is set."""
    con = sqlite3.connect(db)
    agg = "max" if largest else "avg"
    rows = con.execute(f"select kernel_name, counter_name, {agg}(value) from counters_collection "
                       "group by kernel_name, counter_name").fetchall()
    d = collections.defaultdict(dict)
    for kn, cn, v in rows:
        d[kn][cn] = v
    return d


def copy_ref(db, counter):
    """The counter value of the reference copy: the largest copy-kernel
    dispatch of the run (the 512 MiB copy; smaller copies of the program
    itself use the same kernel)."""
    best = 0.0
    for name, v in counters(db, largest=True).items():
        if kind_of(name) == "copy":
            best = max(best, v.get(counter, 0.0))
    return best


def by_kind(cnt, kt, kind):
    """Counters of the kernel instance the trace chose for this kind (the copy
    reference is looked up by kind)."""
    if kind in kt and kt[kind][0] in cnt:
        return cnt[kt[kind][0]]
    for name, v in cnt.items():
        if kind_of(name) == kind:
            return v
    return {}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--sq", default=None)
    ap.add_argument("--size", required=True, help="HxWxC of the profiled workload")
    ap.add_argument("--iters", type=int, default=4, help="N of the profiled workload")
    ap.add_argument("--command", required=True, help="the rocprofv3 command line that produced the data")
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic", default=os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                                      "profiles", "traffic.json"))
    a = ap.parse_args()
    kt = trace(a.trace)
    fe = counters(a.fetch)
    wr = counters(a.write)
    sq = counters(a.sq) if a.sq else {}
    fscale = COPY_BYTES / (copy_ref(a.fetch, "FETCH_SIZE") * 1024.0)
    wscale = COPY_BYTES / (copy_ref(a.write, "WRITE_SIZE") * 1024.0)
    H, W, C = (int(v) for v in a.size.split("x"))
    img = C * H * W * 4
    spec = C * H * (W // 2 + 1) * 8
    alg = {"row_first": img + spec, "row_mid": img + 2 * spec, "row_final": img + spec, "column": 2 * spec}
    lines = [f"# rocprofv3 summary: ILS passes, {W}x{H}x{C} float32, N={a.iters}", "",
             f"command: {a.command}", f"kernel source hash: {source_hash()}",
             f"counter scale from a {COPY_BYTES >> 20} MiB copy: FETCH_SIZE x{fscale:.4f}, WRITE_SIZE x{wscale:.4f}",
             "", f"{'pass':10s} {'calls':>5s} {'avg_us':>8s} {'min_us':>8s} {'max_us':>8s} "
                 f"{'alg_MB':>8s} {'hbm_MB':>8s} {'rd_MB':>8s} {'wr_MB':>8s} {'alg_GB/s':>9s} {'hbm_GB/s':>9s}"]
    traffic = {}
    if os.path.exists(a.traffic):
        with open(a.traffic) as fh:
            traffic = json.load(fh)
    for k in ("row_first", "row_mid", "column", "row_final"):
        if k not in kt:
            continue
        name, calls, avg, lo, hi = kt[k]
        rd = by_kind(fe, kt, k).get("FETCH_SIZE", 0.0) * 1024 * fscale
        wb = by_kind(wr, kt, k).get("WRITE_SIZE", 0.0) * 1024 * wscale
        lines.append(f"{k:10s} {calls:5d} {avg:8.3f} {lo:8.3f} {hi:8.3f} {alg[k] / 1e6:8.2f} {(rd + wb) / 1e6:8.2f} "
                     f"{rd / 1e6:8.2f} {wb / 1e6:8.2f} {alg[k] / (avg * 1e3):9.1f} {(rd + wb) / (avg * 1e3):9.1f}")
        traffic[f"{k}@{a.size}"] = {"bytes_per_launch": int(rd + wb), "read_bytes": int(rd), "write_bytes": int(wb),
                                    "source_hash": source_hash(), "kernel": name}
    tl = timeline(a.trace, kt, 2 * a.iters + 1)
    if tl:
        span, busy, gaps, n = tl
        lines += ["", f"steps in the trace: {n} whole sequences of {2 * a.iters + 1} launches; per step (medians): "
                      f"first start to last end {span:.2f} us, kernel durations {busy:.2f} us, "
                      f"gaps between launches {gaps:.2f} us"]
    if sq:
        lines += ["", "SQ counters per launch (SQ_INSTS_* and SQ_WAVES per dispatch; cycles summed over SQs):"]
        for k in ("row_first", "row_mid", "column", "row_final"):
            sk = by_kind(sq, kt, k)
            if sk:
                lines.append(f"  {k}: " + ", ".join(f"{cn}={v:.0f}" for cn, v in sorted(sk.items())))
                traffic.setdefault(f"{k}@{a.size}", {})["sq"] = dict(sk)
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(a.traffic, "w") as fh:
        json.dump(traffic, fh, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
