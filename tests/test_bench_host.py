"""Host logic of bench.py on the CPU: the one-GPU contract, the traffic
records built from rocprofv3 counter files, their source-digest gate, and the
roofline arithmetic."""

import csv
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kern, counter, value in rows:
            w.writerow({"Kernel_Name": kern, "Counter_Name": counter, "Counter_Value": value})
    return path


def test_traffic_record_scales_counters_by_the_copy_kernel(tmp_path, monkeypatch):
    kern = "void hc::(anonymous namespace)::shade_latent_kernel<2, false, true>(...)"
    copy = "__amd_rocclr_copyBuffer"
    d = str(tmp_path)
    fetch = _counter_csv(os.path.join(d, "fetch"), [(kern, "FETCH_SIZE", 1000.0), (kern, "FETCH_SIZE", 3000.0),
                                                    ("other", "FETCH_SIZE", 9e9)])
    write = _counter_csv(os.path.join(d, "write"), [(kern, "WRITE_SIZE", 64.0)])
    cfetch = _counter_csv(os.path.join(d, "cf"), [(copy, "FETCH_SIZE", float(1 << 19))])   # half of 1 GiB
    cwrite = _counter_csv(os.path.join(d, "cw"), [(copy, "WRITE_SIZE", float(1 << 20))])
    req = _counter_csv(os.path.join(d, "req"), [(kern, "TCC_EA0_RDREQ_sum", 10.0),
                                                (kern, "TCC_EA0_RDREQ_128B_sum", 8.0),
                                                (kern, "TCC_EA0_RDREQ_DRAM_sum", 6.0)])
    out = os.path.join(d, "record.json")
    monkeypatch.setattr(bench, "TRAFFIC_JSON", out)
    bench.record_traffic(fetch, write, cfetch, cwrite, req)
    rec = json.load(open(out))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["fetch_bytes_per_launch"] == 2000.0 * 1024 * 2.0     # mean of the kernel's rows only
    assert rec["write_bytes_per_launch"] == 64.0 * 1024
    assert rec["fetch_plus_write_bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    assert rec["ea_read_bytes"] == 8.0 * 128 and rec["dram_read_bytes"] == 6.0 * 128
    assert rec["kernel_source_sha"] == bench.kernel_source_sha()
    # the gate: the record counts while the digest matches the sources, not after
    assert bench.measured_traffic()["fetch_bytes_per_launch"] == rec["fetch_bytes_per_launch"]
    rec["kernel_source_sha"] = "0" * 16
    json.dump(rec, open(out, "w"))
    assert bench.measured_traffic() is None


def test_stress_record_goes_to_its_own_file(tmp_path, monkeypatch):
    kern = "shade_latent_kernel<3, true, true>"
    d = str(tmp_path)
    fetch = _counter_csv(os.path.join(d, "f"), [(kern, "FETCH_SIZE", 10.0)])
    write = _counter_csv(os.path.join(d, "w"), [(kern, "WRITE_SIZE", 1.0)])
    cf = _counter_csv(os.path.join(d, "cf"), [("__amd_rocclr_copyBuffer", "FETCH_SIZE", float(1 << 20))])
    cw = _counter_csv(os.path.join(d, "cw"), [("__amd_rocclr_copyBuffer", "WRITE_SIZE", float(1 << 20))])
    main, stress = os.path.join(d, "main.json"), os.path.join(d, "stress.json")
    monkeypatch.setattr(bench, "TRAFFIC_JSON", main)
    monkeypatch.setattr(bench, "TRAFFIC_STRESS_JSON", stress)
    bench.record_traffic(fetch, write, cf, cw, stress=True)
    assert os.path.exists(stress) and not os.path.exists(main)
    rec = json.load(open(stress))
    assert rec["workload"] == bench.STRESS and "ea_read_bytes" not in rec
    assert bench.measured_traffic(stress=True) is not None and bench.measured_traffic() is None


def test_missing_counter_rows_stop_the_record(tmp_path, monkeypatch):
    d = str(tmp_path)
    empty = _counter_csv(os.path.join(d, "e"), [("other_kernel", "FETCH_SIZE", 1.0)])
    cf = _counter_csv(os.path.join(d, "cf"), [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 1.0)])
    monkeypatch.setattr(bench, "TRAFFIC_JSON", os.path.join(d, "x.json"))
    with pytest.raises(SystemExit):
        bench.record_traffic(empty, empty, cf, cf)


def test_roofline_and_traffic_arithmetic():
    ceiling = {"rows_per_s": 50e9}
    roof = bench.frame_roofline("k", 4e9, 2e-3, 80e6, ceiling, 5000.0, "lines")
    assert roof["achieved"] == pytest.approx(2000.0)          # 4 GB in 2 ms
    assert roof["frac"] == pytest.approx(2000.0 / bench.HBM_PEAK_GBS)
    assert roof["path_vertices_per_s"] == pytest.approx(40e9)
    assert roof["frac_of_gather_ceiling"] == pytest.approx(0.8)
    assert roof["frac_of_copy"] == pytest.approx(0.4)
    bench.attach_traffic(roof, None, 2e-3)
    assert roof["traffic"] is None and "traffic_GBs" not in roof
    rec = {"fetch_plus_write_bytes_per_launch": 10e9, "note": "n", "fetch_bytes_per_launch": 9e9}
    bench.attach_traffic(roof, rec, 2e-3)
    assert roof["traffic"] == 10e9 and roof["traffic_GBs"] == pytest.approx(5000.0)
    assert roof["traffic_fetch_bytes_per_launch"] == 9e9 and roof["traffic_dram_read_bytes"] is None


def test_committed_records_name_their_workloads():
    for path, workload in ((bench.TRAFFIC_JSON, bench.WORKLOAD), (bench.TRAFFIC_STRESS_JSON, bench.STRESS)):
        rec = json.load(open(path))
        assert rec["workload"] == workload
        assert len(rec["kernel_source_sha"]) == 16
        assert rec["fetch_plus_write_bytes_per_launch"] > 0
