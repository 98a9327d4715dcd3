"""Benchmark and profile-summary plumbing (CPU): bench.py refuses more than
one GPU before touching one, and the rocprofv3 summarisers read counter CSVs
as bench.py and the committed profiles expect."""
import csv
import os
import subprocess
import sys

from paper_2605_08699_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_counters_average_per_kernel(tmp_path):
    a = tmp_path / "a.csv"
    # two dispatches of k_x (one counter split over two dimensions in the
    # first), one of k_y, and a kernel the match leaves out
    _counter_csv(a, [(1, "tigas::k_x(int)", "VALUBusy", 40.0), (1, "tigas::k_x(int)", "SQ_WAVES", 3.0),
                     (1, "tigas::k_x(int)", "SQ_WAVES", 5.0), (2, "tigas::k_x(int)", "VALUBusy", 60.0),
                     (2, "tigas::k_x(int)", "SQ_WAVES", 8.0), (3, "tigas::k_y(int)", "VALUBusy", 10.0),
                     (4, "other(int)", "VALUBusy", 99.0)])
    out = tmp_path / "c.md"
    profiling.counters([(str(a), "cmd a")], str(out), "tigas::", "t")
    rows = {tuple(c.strip() for c in line.split("|")[1:3]): line.split("|")
            for line in out.read_text().splitlines() if line.startswith("| `")}
    assert float(rows[("`tigas::k_x`", "VALUBusy")][4]) == 50.0
    assert float(rows[("`tigas::k_x`", "SQ_WAVES")][4]) == 8.0
    assert int(rows[("`tigas::k_x`", "SQ_WAVES")][3]) == 2
    assert float(rows[("`tigas::k_y`", "VALUBusy")][4]) == 10.0
    assert not any("other" in k[0] for k in rows)
    assert "cmd a" in out.read_text()


def test_traffic_round_trip(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    n = 1 << 20
    # the copies read n/2 KiB on FETCH_SIZE and n KiB on WRITE_SIZE for n KiB
    # moved: scale factors 2 and 1
    _counter_csv(fetch, [(1, copy, "FETCH_SIZE", n / 1024 / 2), (2, "tigas::k_z(int)", "FETCH_SIZE", 100.0),
                         (3, "tigas::k_z(int)", "FETCH_SIZE", 300.0)])
    _counter_csv(write, [(1, copy, "WRITE_SIZE", n / 1024), (2, "tigas::k_z(int)", "WRITE_SIZE", 50.0),
                         (3, "tigas::k_z(int)", "WRITE_SIZE", 50.0)])
    out = tmp_path / "t.md"
    profiling.traffic(str(fetch), str(write), str(out), "fc", "wc", n)
    sha, t = profiling.read_traffic(str(out))
    assert sha == profiling.source_sha1()
    # mean fetch 200 KiB x 2 + mean write 50 KiB x 1 per launch
    assert abs(t["tigas::k_z(int)"] - (200 * 2 + 50) * 1024) < 1e-6
