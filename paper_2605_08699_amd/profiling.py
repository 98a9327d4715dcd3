"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2605_08699_amd.profiling stats KERNEL_STATS_CSV OUT_MD --command CMD [--title T]
    python -m paper_2605_08699_amd.profiling traffic OUT_MD --fetch CSV CMD [--fetch CSV CMD ...]
        --write CSV CMD [--write CSV CMD ...] [--copy-bytes N]
    python -m paper_2605_08699_amd.profiling launches KERNEL_TRACE_CSV OUT_MD --match SUBSTR --command CMD
        [--title T]
    python -m paper_2605_08699_amd.profiling bandwidth TRAFFIC_MD OUT_MD --stats KERNEL_STATS_CSV [--stats ...]
        [--lds COUNTER_CSV] [--command CMD ...] [--title T]
    python -m paper_2605_08699_amd.profiling counters OUT_MD --run CSV CMD [--run CSV CMD ...] --match SUBSTR
        [--title T]

`stats` turns a `--kernel-trace --stats` kernel_stats.csv into a table.
`launches` groups the dispatches of the kernels whose name contains SUBSTR
in a kernel_trace.csv by (kernel, workgroups): one launch shape per frame
size, so sizes that share a kernel get a row each.
`counters` averages, per kernel whose name contains SUBSTR, every counter of
one or more `--pmc` counter_collection CSVs over that kernel's dispatches.
`bandwidth` divides each kernel's HBM bytes per launch (a `traffic` summary)
and LDS bytes per launch (a `--pmc SQ_LDS_IDX_ACTIVE SQ_LDS_BANK_CONFLICT`
CSV) by its average launch time (kernel_stats CSVs) and sets them against the
HBM and LDS peaks.
`traffic` turns `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` counter_collection
CSVs (one pair per run) into HBM bytes per launch of every kernel.  The counters are scaled by
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
    """fetch_csv / write_csv / fetch_cmd / write_cmd: one run each, or lists of
    runs (say the same workload with two tile configurations); each run is
    calibrated against its own copies, and a kernel's bytes per launch are
    averaged over its dispatches in every run."""
    as_list = lambda x: [x] if isinstance(x, str) else list(x)
    fetch_csv, write_csv = as_list(fetch_csv), as_list(write_csv)
    fetch_cmd, write_cmd = as_list(fetch_cmd), as_list(write_cmd)
    acc = collections.defaultdict(lambda: [0, 0.0, 0, 0.0])
    cal = []
    for fpath, wpath in zip(fetch_csv, write_csv):
        fd, wd = per_dispatch(fpath), per_dispatch(wpath)
        ff, fn, fk = calibration(fd, copy_bytes)
        wf, wn, wk = calibration(wd, copy_bytes)
        cal.append((ff, fn, fk, wf, wk))
        for n, v in fd.values():
            a = acc[n]
            a[0] += 1
            a[1] += v * 1024.0 * ff
        for n, v in wd.values():
            a = acc[n]
            a[2] += 1
            a[3] += v * 1024.0 * wf
    rows = []
    for n, (cf, sf, cw, sw) in acc.items():
        if n.startswith(COPY_KERNEL) or not cf or not cw:
            continue
        fb = sf / cf
        wb = sw / cw
        rows.append((fb + wb, n, cf, fb, wb))
    rows.sort(reverse=True)
    with open(dst, "w") as f:
        f.write("# HBM traffic per launch: 3M Gaussians, 1920x1080, FP32 attributes\n\n")
        f.write("Commands (run from the repository root on one MI355X, one counter per run):\n\n```\n")
        for fc, wc in zip(fetch_cmd, write_cmd):
            f.write(f"{fc}\n{wc}\n")
        f.write("```\n\n")
        for ff, fn, fk, wf, wk in cal:
            f.write(f"Calibration: bench.py copies {copy_bytes} bytes device to device; for those copies "
                    f"({fn} dispatches) FETCH_SIZE reads {fk:.0f} KiB and WRITE_SIZE reads {wk:.0f} KiB, so the "
                    f"counters are scaled by {ff:.3f} (fetch) and {wf:.3f} (write).\n\n")
        f.write("| kernel | launches | fetch MB | write MB | total MB per launch |\n|---|---:|---:|---:|---:|\n")
        for tot, n, c, fb, wb in rows:
            f.write(f"| `{short(n)}` | {c} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {tot / 1e6:.1f} |\n")
        f.write(f"\nMachine-readable (bench.py uses a line only while the kernel source is unchanged):\n\n```\n"
                f"kernel_source_sha1 = {source_sha1()}\n")
        for tot, n, c, fb, wb in rows:
            f.write(f"traffic_bytes_per_launch[{n}] = {tot:.0f}\n")
        f.write("```\n")


HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# LDS: 32 banks x 4 bytes per clock per compute unit, 256 compute units, 2.4 GHz
LDS_BYTES_PER_CLOCK = 128
LDS_PEAK_GBS = LDS_BYTES_PER_CLOCK * 256 * 2.4


def bandwidth(traffic_md, stats_csvs, lds_csv, dst, title, commands):
    """Per kernel: HBM bytes per launch (the traffic summary) and LDS bytes
    per launch ((SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT) cycles, summed over
    the compute units, x 128 bytes: the cycles the LDS moves data for indexed
    operations, bank-conflict stalls excluded), each divided by the kernel's
    average launch duration from kernel_stats CSVs, against the peaks."""
    _sha, hbm = read_traffic(traffic_md)
    dur = {}
    for path in stats_csvs:
        for r in csv.DictReader(open(path)):
            dur[r["Name"]] = float(r["AverageNs"]) * 1e-9
    lds = collections.defaultdict(lambda: [0, 0.0])
    per = collections.defaultdict(float)
    if lds_csv:
        for r in csv.DictReader(open(lds_csv)):
            if r["Counter_Name"] in ("SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT"):
                sign = 1.0 if r["Counter_Name"] == "SQ_LDS_IDX_ACTIVE" else -1.0
                per[(int(r["Dispatch_Id"]), r["Kernel_Name"])] += sign * float(r["Counter_Value"])
        for (_d, name), cyc in per.items():
            lds[name][0] += 1
            lds[name][1] += cyc * LDS_BYTES_PER_CLOCK
    rows = []
    for name, sec in dur.items():
        if name not in hbm and name not in lds:
            continue
        hb = hbm.get(name)
        lb = lds[name][1] / lds[name][0] if name in lds else None
        rows.append((-(hb or 0.0) / sec, name, sec, hb, lb))
    rows.sort()
    with open(dst, "w") as f:
        f.write(f"# {title}\n\nInputs (run from the repository root on one MI355X):\n\n```\n")
        for c in commands:
            f.write(c + "\n")
        f.write(f"```\n\nPeaks: HBM {HBM_PEAK_GBS:.0f} GB/s; LDS {LDS_BYTES_PER_CLOCK} B per clock per compute unit x "
                f"256 x 2.4 GHz = {LDS_PEAK_GBS:.0f} GB/s.\n\n")
        f.write("| kernel | avg us | HBM MB per launch | HBM GB/s | of HBM peak | LDS MB per launch | LDS GB/s | "
                "of LDS peak |\n|---|---:|---:|---:|---:|---:|---:|---:|\n")
        for _k, name, sec, hb, lb in rows:
            hcol = f"{hb / 1e6:.1f} | {hb / sec / 1e9:.0f} | {hb / sec / 1e9 / HBM_PEAK_GBS:.3f}" if hb else "- | - | -"
            lcol = (f"{lb / 1e6:.1f} | {lb / sec / 1e9:.0f} | {lb / sec / 1e9 / LDS_PEAK_GBS:.3f}"
                    if lb is not None else "- | - | -")
            f.write(f"| `{short(name)}` | {sec * 1e6:.1f} | {hcol} | {lcol} |\n")


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
    b.add_argument("dst")
    b.add_argument("--fetch", nargs=2, action="append", required=True, metavar=("CSV", "CMD"))
    b.add_argument("--write", nargs=2, action="append", required=True, metavar=("CSV", "CMD"))
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
    g = sub.add_parser("bandwidth")
    g.add_argument("traffic_md")
    g.add_argument("dst")
    g.add_argument("--stats", action="append", required=True)
    g.add_argument("--lds", default=None)
    g.add_argument("--command", action="append", default=[])
    g.add_argument("--title", default="Achieved HBM and LDS bandwidth per kernel")
    args = ap.parse_args()
    if args.cmd == "bandwidth":
        bandwidth(args.traffic_md, args.stats, args.lds, args.dst, args.title, args.command)
    elif args.cmd == "counters":
        counters(args.run, args.dst, args.match, args.title)
    elif args.cmd == "stats":
        stats(args.src, args.dst, args.command, args.title)
    elif args.cmd == "launches":
        launches(args.src, args.dst, args.match, args.command, args.title)
    else:
        traffic([c for c, _ in args.fetch], [c for c, _ in args.write], args.dst,
                [m for _, m in args.fetch], [m for _, m in args.write], args.copy_bytes)


if __name__ == "__main__":
    main()
