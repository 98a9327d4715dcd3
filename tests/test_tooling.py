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


def test_traffic_over_two_runs_calibrates_each_run_on_its_own_copies(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    n = 1 << 20
    f1, w1, f2, w2 = (tmp_path / x for x in ("f1.csv", "w1.csv", "f2.csv", "w2.csv"))
    # run 1 scales fetch by 2, run 2 by 4; k_z runs in both, k_a only in run 2
    _counter_csv(f1, [(1, copy, "FETCH_SIZE", n / 1024 / 2), (2, "tigas::k_z(int)", "FETCH_SIZE", 100.0)])
    _counter_csv(w1, [(1, copy, "WRITE_SIZE", n / 1024), (2, "tigas::k_z(int)", "WRITE_SIZE", 10.0)])
    _counter_csv(f2, [(1, copy, "FETCH_SIZE", n / 1024 / 4), (2, "tigas::k_z(int)", "FETCH_SIZE", 100.0),
                      (3, "tigas::k_a(int)", "FETCH_SIZE", 7.0)])
    _counter_csv(w2, [(1, copy, "WRITE_SIZE", n / 1024), (2, "tigas::k_z(int)", "WRITE_SIZE", 30.0),
                      (3, "tigas::k_a(int)", "WRITE_SIZE", 1.0)])
    out = tmp_path / "t.md"
    profiling.traffic([str(f1), str(f2)], [str(w1), str(w2)], str(out), ["fc1", "fc2"], ["wc1", "wc2"], n)
    _sha, t = profiling.read_traffic(str(out))
    assert abs(t["tigas::k_z(int)"] - ((100 * 2 + 100 * 4) / 2 + (10 + 30) / 2) * 1024) < 1e-6
    assert abs(t["tigas::k_a(int)"] - (7 * 4 + 1) * 1024) < 1e-6
    text = out.read_text()
    assert all(c in text for c in ("fc1", "fc2", "wc1", "wc2")) and text.count("Calibration:") == 2


def test_bandwidth_divides_bytes_by_launch_time(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    n = 1 << 20
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fetch, [(1, copy, "FETCH_SIZE", n / 1024), (2, "tigas::k_z(int)", "FETCH_SIZE", 1000.0)])
    _counter_csv(write, [(1, copy, "WRITE_SIZE", n / 1024), (2, "tigas::k_z(int)", "WRITE_SIZE", 0.0)])
    tmd = tmp_path / "t.md"
    profiling.traffic(str(fetch), str(write), str(tmd), "fc", "wc", n)
    stats = tmp_path / "s.csv"
    with open(stats, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "AverageNs"])
        w.writerow(["tigas::k_z(int)", 3, 1024.0])  # 1000 KiB in 1.024 us: 1e12 B/s
    lds = tmp_path / "l.csv"
    # two dispatches: (100 - 20) and (60 - 0) active cycles over the CUs
    _counter_csv(lds, [(1, "tigas::k_z(int)", "SQ_LDS_IDX_ACTIVE", 100.0),
                       (1, "tigas::k_z(int)", "SQ_LDS_BANK_CONFLICT", 20.0),
                       (2, "tigas::k_z(int)", "SQ_LDS_IDX_ACTIVE", 60.0),
                       (2, "tigas::k_z(int)", "SQ_INSTS_LDS", 5.0)])
    out = tmp_path / "b.md"
    profiling.bandwidth(str(tmd), [str(stats)], str(lds), str(out), "t", ["cmd"])
    row = [l for l in out.read_text().splitlines() if l.startswith("| `tigas::k_z`")][0].split(" | ")
    assert row[1] == "1.0" and row[3] == "1000" and row[4] == "0.125"  # 1000 GB/s of 8000
    lds_bytes = (80 + 60) / 2 * profiling.LDS_BYTES_PER_CLOCK
    assert abs(float(row[6]) - round(lds_bytes / 1.024e-6 / 1e9)) <= 1


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)  # no GPU work: main() runs only as a script
    return mod


def test_roofline_picks_the_blend_and_counts_its_work_per_launch():
    """The roofline line of the FP32 run: the costliest kernel with a work
    model is the blend (ALU-bound), its flops are 12 per evaluation and 9 per
    contribution, per launch, divided by the average launch time."""
    b = _bench_module()
    work = dict(frames=2, visible=2 * 1.5e6, duplicates=2 * 6e6, evaluations=2 * 2e8, contributions=2 * 1.2e8,
                fallbacks=0)
    kernels = {
        "void tigas::k_blend<16, 32, 1, 1, false>(tigas::BlendArgs)":
            dict(launches_per_frame=1.0, avg_us=150.0, ms_per_frame=0.150),
        "void tigas::k_preprocess<0, 3>(tigas::SceneView, ...)": dict(launches_per_frame=1.0, avg_us=133.0,
                                                                      ms_per_frame=0.133),
        "void tigas::k_sort_downsweep<true, false, 512, 512>(unsigned int const*, ...)":
            dict(launches_per_frame=3.0, avg_us=19.0, ms_per_frame=0.057),
    }
    r = b.roofline(dict(work=work, kernels=kernels, sort_passes=4), 3_000_000, "f32")
    assert r["bound"] == "alu" and "k_blend" in r["kernel"]
    flops = 12 * 2e8 + 9 * 1.2e8
    assert abs(r["achieved"] - flops / 150e-6 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 157.3) < 1e-12


def test_depth_pass_bytes_follow_the_three_pass_kernel_names():
    """Three 9-bit depth passes (kernel named with 512 digits and 512
    threads) move 24 bytes per visible Gaussian each; the tile passes of the
    radix path 16 bytes per duplicate each."""
    b = _bench_module()
    w = dict(frames=1, visible=1e6, duplicates=5e6, evaluations=0, contributions=0)
    bound, amount = b.kernel_work("void tigas::k_sort_downsweep<true, false, 512, 512>(...)", w, 3e6, "f32", 0)
    assert bound == "hbm" and amount == 3 * 24 * 1e6
    bound, amount = b.kernel_work("void tigas::k_sort_downsweep<true, false, 256, 256>(...)", w, 3e6, "f32", 0)
    assert amount == 4 * 24 * 1e6
    bound, amount = b.kernel_work("void tigas::k_sort_downsweep<false, false, 256, 256>(...)", w, 3e6, "f32", 2)
    assert amount == 2 * 16 * 5e6
