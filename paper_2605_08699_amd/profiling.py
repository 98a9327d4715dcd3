"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2605_08699_amd.profiling stats KERNEL_STATS_CSV OUT_MD --command CMD [--title T]
    python -m paper_2605_08699_amd.profiling traffic FETCH_CSV WRITE_CSV OUT_MD --fetch-command CMD
        --write-command CMD [--copy-bytes N]
    python -m paper_2605_08699_amd.profiling launches KERNEL_TRACE_CSV OUT_MD --match SUBSTR --command CMD
        [--title T]
    python -m paper_2605_08699_amd.profiling counters OUT_MD --run CSV CMD [--run CSV CMD ...] --match SUBSTR
        [--title T]

`stats` turns a `--kernel-trace --stats` kernel_stats.csv into a table.
`launches` groups the dispatches of the kernels whose name contains SUBSTR
in a kernel_trace.csv by (kernel, workgroups): one launch shape per frame
size, so sizes that share a kernel get a row each.
`counters` averages, per kernel whose name contains SUBSTR, every counter of
one or more `--pmc` counter_collection CSVs over that kernel's dispatches.
`traffic` turns two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` counter_collection
CSVs into HBM bytes per launch of every kernel.  The counters are scaled by
what they read for the plain device-to-device copies of known size that
bench.py makes (the largest `__amd_rocclr_copyBuffer` dispatches): a copy of N
bytes reads N and writes N bytes.  The output carries one machine-readable
line per kernel (`traffic_bytes_per_launch[NAME] = B`) and the SHA-1 of the
kernel source it was measured on, which bench.py checks before using it.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCE = os.path.join(ROOT, "paper_2605_08699_amd", "csrc", "kernels.hip")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def source_sha1() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def short(name: str) -> str:
    return name[:name.index("(")] if "(" in name else name


def stats(src, dst, command, title):
    rows = list(csv.DictReader(open(src)))
    with open(dst, "w") as f:
        f.write(f"# {title}\n\nCommand (run from the repository root on one MI355X):\n\n```\n{command}\n```\n\n")
        f.write("| kernel | calls | avg us | min us | max us | % of GPU time |\n|---|---:|---:|---:|---:|---:|\n")
        for r in rows:
            name = short(r["Name"]).replace("|", "/")
            f.write(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                    f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |\n")


def launches(src, dst, match, command, title):
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(src)):
        n = r["Kernel_Name"]
        if match not in n:
            continue
        wg = int(r["Grid_Size_X"]) // max(int(r["Workgroup_Size_X"]), 1)
        acc[(short(n), wg)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    with open(dst, "w") as f:
        f.write(f"# {title}\n\nCommand (run from the repository root on one MI355X):\n\n```\n{command}\n```\n\n")
        f.write("| kernel | workgroups | launches | avg us | min us | max us |\n|---|---:|---:|---:|---:|---:|\n")
        for (n, wg), ts in sorted(acc.items(), key=lambda kv: (kv[0][1], kv[0][0])):
            f.write(f"| `{n}` | {wg} | {len(ts)} | {sum(ts) / len(ts):.1f} | {min(ts):.1f} | {max(ts):.1f} |\n")


def per_dispatch(path):
    """{dispatch id: (kernel name, counter value summed over the dimensions)}"""
    d = {}
    for r in csv.DictReader(open(path)):
        k = int(r["Dispatch_Id"])
        name, v = d.get(k, (r["Kernel_Name"], 0.0))
        d[k] = (name, v + float(r["Counter_Value"]))
    return d


def counters(runs, dst, match, title):
    """Per (kernel, counter): the mean over dispatches of the counter's value
    (summed over its dimensions within a dispatch)."""
    acc = collections.defaultdict(lambda: [0, 0.0])
    order = []
    for path, _cmd in runs:
        per = collections.defaultdict(float)  # (dispatch, kernel, counter) -> value
        for r in csv.DictReader(open(path)):
            if match not in r["Kernel_Name"]:
                continue
            per[(int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"])] += float(r["Counter_Value"])
        for (_d, name, ctr), v in per.items():
            key = (short(name).replace("|", "/"), ctr)
            if key not in acc:
                order.append(key)
            acc[key][0] += 1
            acc[key][1] += v
    with open(dst, "w") as f:
        f.write(f"# {title}\n\nCommands (run from the repository root on one MI355X, one counter set per run):\n\n```\n")
        for _path, cmd in runs:
            f.write(cmd + "\n")
        f.write("```\n\n| kernel | counter | dispatches | mean per dispatch |\n|---|---|---:|---:|\n")
        for key in sorted(order):
            n, v = acc[key]
            f.write(f"| `{key[0]}` | {key[1]} | {n} | {v / n:.6g} |\n")


def calibration(d, copy_bytes):
    vals = sorted((v for n, v in d.values() if n.startswith(COPY_KERNEL)), reverse=True)
    if not vals:
        raise SystemExit("no copy dispatch to calibrate against")
    top = [v for v in vals if v > 0.5 * vals[0]]
    top.sort()
    kib = top[len(top) // 2]
    return copy_bytes / (kib * 1024.0), len(top), kib


def traffic(fetch_csv, write_csv, dst, fetch_cmd, write_cmd, copy_bytes):
    fd, wd = per_dispatch(fetch_csv), per_dispatch(write_csv)
    ff, fn, fk = calibration(fd, copy_bytes)
    wf, wn, wk = calibration(wd, copy_bytes)
    acc = collections.defaultdict(lambda: [0, 0.0, 0, 0.0])
    for n, v in fd.values():
        a = acc[n]
        a[0] += 1
        a[1] += v
    for n, v in wd.values():
        a = acc[n]
        a[2] += 1
        a[3] += v
    rows = []
    for n, (cf, sf, cw, sw) in acc.items():
        if n.startswith(COPY_KERNEL) or not cf or not cw:
            continue
        fb = sf / cf * 1024.0 * ff
        wb = sw / cw * 1024.0 * wf
        rows.append((fb + wb, n, cf, fb, wb))
    rows.sort(reverse=True)
    with open(dst, "w") as f:
        f.write("# HBM traffic per launch: 3M Gaussians, 1920x1080, FP32 attributes\n\n")
        f.write("Commands (run from the repository root on one MI355X, one counter per run):\n\n")
        f.write(f"```\n{fetch_cmd}\n{write_cmd}\n```\n\n")
        f.write(f"Calibration: bench.py copies {copy_bytes} bytes device to device; for those copies "
                f"({fn} dispatches) FETCH_SIZE reads {fk:.0f} KiB and WRITE_SIZE reads {wk:.0f} KiB, so the counters "
                f"are scaled by {ff:.3f} (fetch) and {wf:.3f} (write).\n\n")
        f.write("| kernel | launches | fetch MB | write MB | total MB per launch |\n|---|---:|---:|---:|---:|\n")
        for tot, n, c, fb, wb in rows:
            f.write(f"| `{short(n)}` | {c} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {tot / 1e6:.1f} |\n")
        f.write(f"\nMachine-readable (bench.py uses a line only while the kernel source is unchanged):\n\n```\n"
                f"kernel_source_sha1 = {source_sha1()}\n")
        for tot, n, c, fb, wb in rows:
            f.write(f"traffic_bytes_per_launch[{n}] = {tot:.0f}\n")
        f.write("```\n")


def read_traffic(path):
    """(sha1, {kernel name: bytes per launch}) from a file written by `traffic`."""
    sha, t = None, {}
    if not os.path.exists(path):
        return sha, t
    for line in open(path):
        line = line.strip()
        if line.startswith("kernel_source_sha1 = "):
            sha = line.split("= ", 1)[1]
        elif line.startswith("traffic_bytes_per_launch["):
            name, val = line[len("traffic_bytes_per_launch["):].rsplit("] = ", 1)
            t[name] = float(val)
    return sha, t


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("src")
    a.add_argument("dst")
    a.add_argument("--command", required=True)
    a.add_argument("--title", default="rocprofv3 kernel statistics")
    b = sub.add_parser("traffic")
    b.add_argument("fetch")
    b.add_argument("write")
    b.add_argument("dst")
    b.add_argument("--fetch-command", required=True)
    b.add_argument("--write-command", required=True)
    b.add_argument("--copy-bytes", type=int, default=1 << 30)
    c = sub.add_parser("launches")
    c.add_argument("src")
    c.add_argument("dst")
    c.add_argument("--match", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--title", default="rocprofv3 launches")
    e = sub.add_parser("counters")
    e.add_argument("dst")
    e.add_argument("--run", nargs=2, action="append", required=True, metavar=("CSV", "CMD"))
    e.add_argument("--match", required=True)
    e.add_argument("--title", default="rocprofv3 counters")
    args = ap.parse_args()
    if args.cmd == "counters":
        counters(args.run, args.dst, args.match, args.title)
    elif args.cmd == "stats":
        stats(args.src, args.dst, args.command, args.title)
    elif args.cmd == "launches":
        launches(args.src, args.dst, args.match, args.command, args.title)
    else:
        traffic(args.fetch, args.write, args.dst, args.fetch_command, args.write_command, args.copy_bytes)


if __name__ == "__main__":
    main()
