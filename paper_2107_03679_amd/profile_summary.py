"""Summaries of rocprofv3 runs of bench.py for profiles/.

Reads, from one output folder of a profiling call:

* ``bench.json``: the bench line of the same build (its ``roofline`` entry names
  the dominant kernel, its per-launch algorithmic bytes and the key under which
  bench.py looks the traffic record up);
* ``prof/run_kernel_trace.csv``: ``rocprofv3 --kernel-trace --stats -f csv``;
* ``pmc_FETCH_SIZE/run_counter_collection.csv`` and
  ``pmc_WRITE_SIZE/run_counter_collection.csv``: one ``--pmc`` pass per counter.

Writes ``profiles/kernels_<workload>.md`` (durations per kernel and launch
shape, HBM bytes per launch) and ``profiles/traffic_<workload>.json`` (the
dominant kernel's HBM bytes per launch, with the hash of the sources it was
built from, which bench.py checks before reporting the figure).

The counters are scaled by what they read for the bench's copy probe, a plain
device-to-device copy of a known size (``--copy-probe`` MiB read and written).

    python -m paper_2107_03679_amd.profile_summary <folder> [--workload blobs512x60]
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# profiling scope name -> HIP kernel (the launch shape of the finest level takes the most time)
HIP_KERNEL = {
    "up_mv_l0": ("k_up_mv2w", "k_up_mv2"), "up_fused_l0": ("k_up_col", "k_up_fused2"),
    "down_fused_l0": ("k_down_col", "k_down_fused2"), "sstep_gram": ("k_sstep_gram",),
    "sstep_matvec": ("k_sstep_matvec",), "x_update": ("k_x_update",), "residual_ff": ("k_residual_ff",),
    "step_fused_l0": ("k_step_col",), "x_update_residual": ("k_x_update_residual2",),
}
# sources the kernels are built from (any change voids a traffic record)
SOURCES = ["paper_2107_03679_amd/csrc/k_multigrid.hip", "paper_2107_03679_amd/csrc/k_krylov.hip",
           "paper_2107_03679_amd/csrc/dev_common.h", "paper_2107_03679_amd/csrc/kernels.h"]
PMC_REGEX = ("k_up_mv2|k_up_fused2|k_down_fused2|k_up_col|k_down_col|k_sstep|k_residual_ff|k_x_update|k_coarse_cycle|"
             "copyBuffer|elementwise")


def commands(workload: str) -> tuple[str, list[str]]:
    base = (f"python3 $R/bench.py --workload {workload} --steps 1 --warmup 0 --no-cpu-baseline --no-learned "
            "--no-vcycle-leg --tune-cache $OUT/tune.jsonl")
    trace = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -f csv -d $OUT/prof -o run "
             f"-- {base}")
    pmc = [(f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc {ctr} --kernel-include-regex \"{PMC_REGEX}\" -f csv "
            f"-d $OUT/pmc_{ctr} -o run -- {base} --no-profile --no-graph") for ctr in ("FETCH_SIZE", "WRITE_SIZE")]
    return trace, pmc


def kernel_name(raw: str) -> str:
    return raw.replace("(anonymous namespace)::", "").split("(")[0]


def sources_sha256(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("folder")
    ap.add_argument("--workload", default="blobs512x60")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"), help="folder of the summary and the record")
    args = ap.parse_args(argv)
    g = args.folder
    with open(os.path.join(g, "bench.json")) as fh:
        bench = json.loads(fh.read().strip().splitlines()[-1])
    roof = bench["roofline"]
    trace = collections.defaultdict(list)
    with open(os.path.join(g, "prof", "run_kernel_trace.csv")) as fh:
        for r in csv.DictReader(fh):
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])  # threads, as Grid_Size
            trace[(kernel_name(r["Kernel_Name"]), grid)].append(
                int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    pmc = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        a = collections.defaultdict(list)
        with open(os.path.join(g, f"pmc_{ctr}", "run_counter_collection.csv")) as fh:
            for r in csv.DictReader(fh):
                a[(kernel_name(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
        pmc[ctr] = a
    # copy calibration: the probe's four copies (one untimed, three timed) are the first
    # dispatches of the largest copyBuffer grid; later copies of that grid move other sizes
    probe = roof["copy_probe"]
    copies = [k for k in pmc["FETCH_SIZE"] if k[0] == "__amd_rocclr_copyBuffer"]
    ck = max(copies, key=lambda k: k[1])
    half_kib = probe["bytes_per_copy"] / 2 / 1024  # bytes read = bytes written = half the probe's count
    fe, wr = pmc["FETCH_SIZE"][ck][:4], pmc["WRITE_SIZE"][ck][:4]
    f_fetch, f_write = half_kib / (sum(fe) / len(fe)), half_kib / (sum(wr) / len(wr))

    def mb(ctr, key, f):
        v = pmc[ctr].get(key, [0.0])
        return f * sum(v) / len(v) * 1024 / 1e6

    hip = HIP_KERNEL[roof["kernel"]]
    cands = [k for k in trace if k[0].split("<")[0].replace("void ", "") in hip]
    dom = max(cands, key=lambda k: sum(trace[k]))  # the launch shape of the solve (the tuner's trials are few)
    trace_cmd, pmc_cmds = commands(args.workload)
    L = [f"# Kernel profile: {args.workload}\n",
         "Commands, run on an MI355X (`R` = the repository root, `OUT` = an output folder, the same for all "
         "three runs, so that the tuned launch shapes of the first are reused); this file and the traffic record "
         "were written by `python3 -m paper_2107_03679_amd.profile_summary $OUT` from the CSV files they leave.\n",
         f"Kernel trace:\n\n```\n{trace_cmd}\n```\n",
         "HBM counters (one run per counter, eager launches):\n\n```\n" + "\n".join(pmc_cmds) + "\n```\n",
         "The traced run is one graph-replayed step plus the profiled (eager) step of bench.py.  Durations per "
         "launch shape (kernel, grid size in threads):\n",
         "| kernel | grid | launches | avg us | total ms |", "|---|---:|---:|---:|---:|"]
    for (name, grid), v in sorted(trace.items(), key=lambda kv: -sum(kv[1]))[:24]:
        L.append(f"| `{name}` | {grid} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | {sum(v) / 1e6:.2f} |")
    d = trace[dom]
    L.append(f"\nDominant kernel (bench.py roofline entry `{roof['kernel']}`): `{dom[0]}`, grid {dom[1]}: "
             f"{sum(d) / len(d) / 1e3:.2f} us per launch in the trace; the in-bench HIP events on the library "
             f"stream measured {roof['avg_launch_us']:.2f} us.\n")
    L.append(f"Counter calibration with the copy probe ({probe['bytes_per_copy'] / 2 ** 21:.0f} MiB read and as much "
             f"written per copy): FETCH_SIZE reads {sum(fe) / len(fe):.0f} KiB (factor {f_fetch:.3f}), WRITE_SIZE "
             f"{sum(wr) / len(wr):.0f} KiB (factor {f_write:.3f}).  HBM bytes per launch = counter x factor:\n")
    L += ["| kernel | grid | fetch MB | write MB |", "|---|---:|---:|---:|"]
    for k in sorted(pmc["FETCH_SIZE"], key=lambda k: -sum(pmc["FETCH_SIZE"][k]))[:14]:
        L.append(f"| `{k[0]}` | {k[1]} | {mb('FETCH_SIZE', k, f_fetch):.1f} | {mb('WRITE_SIZE', k, f_write):.1f} |")
    fetch, write = mb("FETCH_SIZE", dom, f_fetch) * 1e6, mb("WRITE_SIZE", dom, f_write) * 1e6
    L.append(f"\nDominant kernel: {(fetch + write) / 1e6:.1f} MB of HBM traffic per launch against "
             f"{roof['bytes_per_launch'] / 1e6:.1f} MB of algorithmic bytes "
             f"({(fetch + write) / roof['bytes_per_launch']:.2f}x).\n")
    L.append(f"Bench line of the same build: {bench['value']:.1f} {bench['unit']}, {bench['ms_per_step']:.1f} ms per "
             f"step, copy probe {probe['GB/s']:.0f} GB/s.\n")
    out_md = os.path.join(args.out, f"kernels_{args.workload}.md")
    with open(out_md, "w") as fh:
        fh.write("\n".join(L) + "\n")
    rec = {"workload": args.workload, "kernel": roof["kernel"], "config": roof["record_key"], "hip_kernel": dom[0],
           "grid": dom[1], "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "fetch_factor": f_fetch, "write_factor": f_write, "sources": SOURCES,
           "sources_sha256": sources_sha256(SOURCES), "commands": pmc_cmds}
    with open(os.path.join(args.out, f"traffic_{args.workload}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    with open(out_md) as fh:
        print(fh.read())


if __name__ == "__main__":
    main()
