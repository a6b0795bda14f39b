"""Host-side logic of bench.py, on the CPU: the one-GPU guard and the counter
summary that feeds roofline.traffic (synthetic rocprofv3 counter tables)."""
import csv
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", BENCH)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _counter_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for d, k, c, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_summary_scales_counters_by_the_copy(tmp_path):
    kern = "k_lz_project<float, 4, 0, 3>"
    other = "k_lz_update<float, 4, 1, 3>"
    # two dispatches of the kernel, each reported in two counter instances,
    # plus another kernel's rows that must be ignored
    _counter_csv(tmp_path / "kf.csv", [(1, kern, "FETCH_SIZE", 100.0), (1, kern, "FETCH_SIZE", 50.0),
                                       (2, kern, "FETCH_SIZE", 120.0), (2, kern, "FETCH_SIZE", 30.0),
                                       (3, other, "FETCH_SIZE", 9e9)])
    _counter_csv(tmp_path / "kw.csv", [(1, kern, "WRITE_SIZE", 40.0), (2, kern, "WRITE_SIZE", 40.0),
                                       (3, other, "WRITE_SIZE", 9e9)])
    # a 1 GiB copy whose reads the counter sees at half size and writes at full size
    _counter_csv(tmp_path / "cf.csv", [(7, "rsb::(anonymous namespace)::k_hbm_copy(float __vector(4) const*, float __vector(4)*, long)", "FETCH_SIZE", 524288.0)])
    _counter_csv(tmp_path / "cw.csv", [(7, "rsb::(anonymous namespace)::k_hbm_copy(float __vector(4) const*, float __vector(4)*, long)", "WRITE_SIZE", 1048576.0)])
    out = tmp_path / "traffic.txt"
    r = subprocess.run([sys.executable, BENCH, "--traffic-summary",
                        "--workload", "box128x128x64-holes5-2", "--kernel-name", kern, "--fetch-csv", str(tmp_path / "kf.csv"),
                        "--write-csv", str(tmp_path / "kw.csv"),
                        "--copy-fetch-csv", str(tmp_path / "cf.csv"),
                        "--copy-write-csv", str(tmp_path / "cw.csv"), "--out", str(out)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    kv = dict(line.split(":", 1) for line in out.read_text().splitlines()
              if ":" in line and not line.startswith("#"))
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    assert kv["dispatches_fetch"] == "2" and kv["dispatches_write"] == "2"
    assert float(kv["fetch_scale"]) == 2.0 and float(kv["write_scale"]) == 1.0
    # (150 KiB x 2 + 40 KiB x 1) per dispatch
    assert int(kv["hbm_bytes_per_launch"]) == (150 * 2 + 40) * 1024
    assert kv["workload"] == "box128x128x64-holes5-2" and kv["kernel_name"] == kern


def test_stored_traffic_only_for_its_workload_and_sources(tmp_path):
    bench = _bench_module()
    f = tmp_path / "t.txt"
    f.write_text("workload: wl\nkernel: K\nsource_sha256_16: %s\nhbm_bytes_per_launch: 1234\n"
                 % bench.kernel_source_hash())
    bench.TRAFFIC_FILE = str(f)
    assert bench.stored_traffic("wl", "K") == 1234.0
    assert bench.stored_traffic("other", "K") is None
    assert bench.stored_traffic("wl", "other kernel") is None
    f.write_text("workload: wl\nkernel: K\nsource_sha256_16: 0000000000000000\n"
                 "hbm_bytes_per_launch: 1234\n")
    assert bench.stored_traffic("wl", "K") is None


def test_kernel_stats_table_sorted_by_device_time(tmp_path):
    rows = [("void rsb::(anonymous namespace)::k_small<float>(int)", 10, 1.0e6, 1.0e5, 10.0),
            ("void rsb::(anonymous namespace)::k_big<float, 4>(rsb::LzArgs<float>, int)",
             4, 8.0e6, 2.0e6, 80.0),
            ("k_mid", 2, 1.0e6, 5.0e5, 10.0)]
    src = tmp_path / "kernel_stats.csv"
    with open(src, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writerows(rows)
    out = tmp_path / "stats.txt"
    r = subprocess.run([sys.executable, BENCH, "--stats-summary", str(src), "--out", str(out),
                        "--commands", "cmd"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = out.read_text().splitlines()
    assert lines[1] == "# command: cmd"
    assert "10.0 ms device time" in lines[2]
    body = [l.split() for l in lines[4:]]
    assert [b[0] for b in body] == ["k_big<float,", "k_small<float>", "k_mid"]
    assert body[0][-4:] == ["4", "8.00", "2000.0", "80.00"]
