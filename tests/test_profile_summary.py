"""The rocprofv3 summariser on a synthetic output folder: the copy calibration, the
dominant kernel's launch shape and the traffic record that bench.py looks up."""
import csv
import json
import os

from paper_2107_03679_amd import profile_summary as ps


def _csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_summary_calibrates_counters_and_writes_record(tmp_path):
    g = tmp_path / "run"
    key = {"workload": "toy", "rhs": 2, "levels": 3, "restart": 8, "cycle": 3, "krylov": "sstep", "fused_step": 2}
    bench = {"value": 1.0, "unit": "solves/s", "ms_per_step": 2.0,
             "roofline": {"kernel": "up_mv_l0", "avg_launch_us": 10.0, "bytes_per_launch": 1.0e6, "record_key": key,
                          "copy_probe": {"bytes_per_copy": 2 * 2 ** 20, "GB/s": 5000.0}}}
    os.makedirs(g)
    (g / "bench.json").write_text(json.dumps(bench) + "\n")
    name = "void (anonymous namespace)::k_up_mv2<64, 16>(int, VecSet)"
    _csv(str(g / "prof" / "run_kernel_trace.csv"), ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"],
         [[name, 2048, 0, 10000], [name, 2048, 20000, 30000], [name, 256, 0, 5000]])
    # the probe copies 1 MiB each way; the counters read half the fetched bytes, all the written ones
    copy = "__amd_rocclr_copyBuffer(char const*, char*)"
    rows = {"FETCH_SIZE": [[copy, 4096, 512.0]] * 4 + [[copy, 4096, 100.0], [name, 2048, 300.0], [name, 2048, 500.0]],
            "WRITE_SIZE": [[copy, 4096, 1024.0]] * 4 + [[copy, 4096, 100.0], [name, 2048, 200.0], [name, 2048, 200.0]]}
    for ctr, r in rows.items():
        _csv(str(g / f"pmc_{ctr}" / "run_counter_collection.csv"), ["Kernel_Name", "Grid_Size", "Counter_Value"], r)
    out = tmp_path / "profiles"
    os.makedirs(out)
    ps.main([str(g), "--workload", "toy", "--out", str(out)])
    rec = json.loads((out / "traffic_toy.json").read_text())
    assert rec["grid"] == 2048 and rec["config"] == key
    assert abs(rec["fetch_factor"] - 2.0) < 1e-12 and abs(rec["write_factor"] - 1.0) < 1e-12
    assert abs(rec["fetch_bytes_per_launch"] - 2.0 * 400.0 * 1024) < 1e-6
    assert abs(rec["write_bytes_per_launch"] - 200.0 * 1024) < 1e-6
    md = (out / "kernels_toy.md").read_text()
    assert "10.00 us per launch in the trace" in md and "rocprofv3 --pmc FETCH_SIZE" in md
