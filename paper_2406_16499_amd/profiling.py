"""Turn rocprofv3 CSV output into the short text summaries kept under profiles/.

    python -m paper_2406_16499_amd.profiling stats   --csv DIR/run_kernel_stats.csv \
        --cmd "<rocprofv3 command>" --out profiles/<kernel>_<workload>_stats.txt
    python -m paper_2406_16499_amd.profiling traffic --fetch DIR1/run_counter_collection.csv \
        --write DIR2/run_counter_collection.csv --kernel panel_final_y --match "k_panel_final_y<float>" \
        --cmd-fetch "<command>" --cmd-write "<command>" --out profiles/panel_final_y_traffic.txt

`traffic` scales the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) of
the matched kernel by what the same counters read for the calibration copy
(k_copy16, COPY_BYTES read and written), and records the hash of the kernel
sources so that bench.py drops the figure once the kernels change.
"""
from __future__ import annotations

import argparse
import csv
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _short(name: str) -> str:
    """Kernel name without the return type, namespace and parameter list."""
    name = name.replace("void ", "").replace("lsq::", "")
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and i > 0:
            return name[:i]
    return name


def stats_summary(stats_csv: str, command: str, out: str, top: int = 30) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    total = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel statistics", f"# command: {command}", "",
             f"{'kernel':<60} {'calls':>7} {'total_us':>11} {'avg_us':>9} {'min_us':>9} {'max_us':>9} {'pct':>6}"]
    for r in rows[:top]:
        lines.append(f"{_short(r['Name'])[:60]:<60} {int(r['Calls']):>7} "
                     f"{float(r['TotalDurationNs']) / 1e3:>11.1f} {float(r['AverageNs']) / 1e3:>9.2f} "
                     f"{float(r['MinNs']) / 1e3:>9.2f} {float(r['MaxNs']) / 1e3:>9.2f} "
                     f"{100.0 * float(r['TotalDurationNs']) / total:>6.2f}")
    text = "\n".join(lines) + "\n"
    with open(out, "w") as fh:
        fh.write(text)
    return text


def _per_dispatch(path: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter (summed over the
    dimensions rocprofv3 reports it in)."""
    acc = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        acc[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    out = defaultdict(list)
    for key, v in acc.items():
        out[names[key]].append(v)
    return out


def _mean_for(per: dict, match: str):
    """Mean over the dispatches of every kernel whose name contains one of the
    '|'-separated alternatives of match."""
    alts = [m for m in match.split("|") if m]
    vals = [v for name, vs in per.items() if any(m in name for m in alts) for v in vs]
    if not vals:
        raise SystemExit(f"no dispatch of a kernel matching {match!r}")
    return sum(vals) / len(vals), len(vals)


def traffic_summary(fetch_csv: str, write_csv: str, kernel: str, match: str, cmd_fetch: str,
                    cmd_write: str, out: str, sources: str = "qr") -> str:
    sys.path.insert(0, ROOT)
    import bench   # noqa: E402  (source hash and calibration size)
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")
    copy_kib = bench.COPY_BYTES / 1024.0
    cf, ncf = _mean_for(fetch, "k_copy16")
    cw, ncw = _mean_for(write, "k_copy16")
    f_fetch, f_write = copy_kib / cf, copy_kib / cw
    kf, nkf = _mean_for(fetch, match)
    kw, nkw = _mean_for(write, match)
    hbm = (kf * f_fetch + kw * f_write) * 1024.0
    lines = [
        f"# HBM traffic of {match} from rocprofv3 hardware counters",
        f"# fetch command: {cmd_fetch}",
        f"# write command: {cmd_write}",
        f"kernel: {kernel}",
        f"match: {match}",
        f"source_hash: {bench.source_hash(bench.BATCH_SOURCES if sources == 'batch' else None)}",
        f"dispatches_fetch: {nkf}",
        f"dispatches_write: {nkw}",
        f"fetch_kib_per_launch_raw: {kf:.1f}",
        f"write_kib_per_launch_raw: {kw:.1f}",
        f"copy_bytes: {bench.COPY_BYTES}",
        f"copy_fetch_kib_raw: {cf:.1f}",
        f"copy_write_kib_raw: {cw:.1f}",
        f"fetch_scale: {f_fetch:.4f}",
        f"write_scale: {f_write:.4f}",
        f"hbm_bytes_per_launch: {hbm:.0f}",
    ]
    text = "\n".join(lines) + "\n"
    with open(out, "w") as fh:
        fh.write(text)
    return text


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="action", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--cmd", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--top", type=int, default=30)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--match", required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--sources", default="qr", choices=["qr", "batch"],
                   help="source set whose hash the summary records")
    a = ap.parse_args(argv)
    if a.action == "stats":
        print(stats_summary(a.csv, a.cmd, a.out, a.top), end="")
    else:
        print(traffic_summary(a.fetch, a.write, a.kernel, a.match, a.cmd_fetch, a.cmd_write, a.out,
                              a.sources),
              end="")


if __name__ == "__main__":
    main()
