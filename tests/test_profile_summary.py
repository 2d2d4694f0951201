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
    # the solve's launch shape (a 3D grid of 2048 threads) takes the most time; a tuner trial with a
    # larger grid and a smaller shape run less
    _csv(str(g / "prof" / "run_kernel_trace.csv"),
         ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp", "End_Timestamp"],
         [[name, 512, 2, 2, 0, 10000], [name, 512, 2, 2, 20000, 30000], [name, 256, 1, 1, 0, 5000],
          [name, 4096, 1, 1, 0, 12000]])
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


def test_network_layer_table_and_summary(tmp_path):
    """The network profile's FLOP count (2 x taps x cin x cout per output point, levels halving
    with ceil) against a hand sum, and its summary of a synthetic trace (two warm-up and one
    timed application, eight convolution dispatches each, in layer order)."""
    from paper_2107_03679_amd import net_profile as npf

    rows = npf.layer_table(2, 60, 577, npf.shapes_of(2))
    sizes = [577, 289, 145, 73]
    hand = 2 * 9 * 60 * (sizes[0] ** 2 * (4 * 16 + 48 * 16 + 16 * 2) + sizes[1] ** 2 * (16 * 32 + 96 * 32)
                         + sizes[2] ** 2 * (32 * 64 + 128 * 64) + sizes[3] ** 2 * 64 * 64)
    assert sum(r[5] for r in rows) == hand == 890042584320
    rows3 = npf.layer_table(3, 8, 177, npf.shapes_of(3))
    assert [r[3:5] for r in rows3] == [(4, 16), (16, 16), (16, 32), (32, 32), (64, 32), (48, 16), (32, 16), (16, 2)]
    conv = "void (anonymous namespace)::k_conv_lds<1, 8, 32, 0, 2, false>(ConvArgs)"
    trace = [[conv, 0, 1000 * (j + 1)] for j in range(16)] + [[conv, 0, 2000] for _ in range(8)]
    _csv(str(tmp_path / "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)
    npf.main(["summarize", str(tmp_path), "--dim", "2", "--nimg", "60", "--n", "577", "--warmup", "2", "--reps", "1",
              "--out", str(tmp_path)])
    text = (tmp_path / "net_layers_2d_60x577.md").read_text()
    assert "| all | | | | 16.0 |" in text  # the timed application only: 8 layers x 2 us
    assert "net_profile run --dim 2 --nimg 60 --n 577 --warmup 2 --reps 1" in text
