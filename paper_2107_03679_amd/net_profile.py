"""Per-layer profile of the learned preconditioner's forward pass.

Two modes:

    python -m paper_2107_03679_amd.net_profile run --dim 2 --nimg 60 --n 577
        applies a network (seed 1, random normal input) `--warmup` + `--reps`
        times on the GPU; meant to run under
        `rocprofv3 --kernel-trace --stats -f csv -d $OUT -o run -- python3 -m ...`.

    python -m paper_2107_03679_amd.net_profile summarize $OUT --dim 2 --nimg 60 --n 577
        reads $OUT/run_kernel_trace.csv, takes the convolution dispatches of the
        timed applications (eight per application, in the network's layer order),
        and writes profiles/net_layers_<dim>d_<nimg>x<n>.md: per layer the mean
        duration, the useful FLOPs (real channels: 2 x taps x cin x cout per output
        point), their rate against the 2.5 PFLOP/s dense BF16 matrix-core peak, and
        the activation bytes (BF16 in and out) against the 8 TB/s HBM peak.
"""
from __future__ import annotations

import argparse
import collections
import csv
import os
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LAYERS = ["A0", "A1", "A2", "A3", "B2", "B1", "B0", "O"]
LEVEL = [0, 1, 2, 3, 2, 1, 0, 0]
CH = {2: (16, 32, 64, 64), 3: (16, 16, 32, 32)}  # encoder channels per level of the library's networks
MFMA_PEAK = 2500.0  # TFLOP/s, dense BF16
HBM_PEAK = 8000.0   # GB/s


def shapes_of(dim: int):
    """(cin, cout) per layer, in LAYERS order."""
    c = CH[dim]
    return [(4, c[0]), (c[0], c[1]), (c[1], c[2]), (c[2], c[3]), (c[3] + c[2], c[2]), (c[2] + c[1], c[1]),
            (c[1] + c[0], c[0]), (c[0], 2)]


def run(args) -> None:
    import torch

    from . import helm

    net = helm.Net(seed=1, dim=args.dim)
    if [tuple(t) for t in net.shapes] != shapes_of(args.dim):
        raise RuntimeError(f"layer table out of date: library {net.shapes}, table {shapes_of(args.dim)}")
    g = torch.Generator(device="cuda").manual_seed(0)
    shape = (args.nimg,) + (args.n,) * args.dim + (4,)
    x = torch.randn(shape, device="cuda", generator=g)
    for _ in range(args.warmup):
        net.forward(x)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.reps):
        net.forward(x)
    torch.cuda.synchronize()
    print(f"forward {args.dim}D {args.nimg} x {args.n}^{args.dim}: "
          f"{(time.perf_counter() - t) / args.reps * 1e3:.2f} ms per application", flush=True)
    net.close()


def layer_table(dim: int, nimg: int, n: int, shapes):
    """(name, level, points, cin, cout, flops, bytes) per layer; bytes are the BF16 activations
    a layer must read and write (a pooled input at the finer level, an upsampled input at the
    coarser one), FP32 for the output layer's two channels."""
    taps = 27 if dim == 3 else 9
    sizes = [n]
    for _ in range(3):
        sizes.append((sizes[-1] + 1) // 2)
    pts = [nimg * s ** dim for s in sizes]
    ch = [shapes[i][1] for i in range(4)]  # encoder outputs per level
    rows = []
    for i, name in enumerate(LAYERS):
        cin, cout = shapes[i]
        lv = LEVEL[i]
        p = pts[lv]
        flops = 2.0 * taps * cin * cout * p
        if name == "A0":
            rd = 8 * 2 * p  # four channels padded to eight
        elif name.startswith("A"):
            rd = ch[lv - 1] * 2 * pts[lv - 1]
        elif name == "O":
            rd = ch[0] * 2 * p
        else:
            rd = (cin - ch[lv]) * 2 * pts[lv + 1] + ch[lv] * 2 * p
        wr = 2 * 4 * p if name == "O" else cout * 2 * p
        rows.append((name, lv, p, cin, cout, flops, rd + wr))
    return rows


def summarize(args) -> None:
    path = os.path.join(args.folder, "run_kernel_trace.csv")
    convs = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if any(k in r["Kernel_Name"] for k in ("k_conv_lds", "k_conv2c", "k_conv2m", "k_conv3c")):
                convs.append((r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0],
                              int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    napp = len(convs) // len(LAYERS)
    timed = convs[len(LAYERS) * args.warmup:len(LAYERS) * napp]
    per = collections.defaultdict(list)
    kname = {}
    for j, (k, ns) in enumerate(timed):
        per[LAYERS[j % len(LAYERS)]].append(ns)
        kname[LAYERS[j % len(LAYERS)]] = k
    rows = layer_table(args.dim, args.nimg, args.n, shapes_of(args.dim))
    run_cmd = (f"cd /tmp && export TMPDIR=/tmp && cd $R && rocprofv3 --kernel-trace --stats -f csv -d $OUT -o run -- "
               f"python3 -m paper_2107_03679_amd.net_profile run --dim {args.dim} --nimg {args.nimg} --n {args.n} "
               f"--warmup {args.warmup} --reps {args.reps}")
    L = [f"# Network layers: {args.dim}D, {args.nimg} x {args.n}^{args.dim}\n",
         "Command, run on an MI355X (`R` = the repository root, `OUT` = an output folder); this file was written by "
         f"`python3 -m paper_2107_03679_amd.net_profile summarize $OUT --dim {args.dim} --nimg {args.nimg} "
         f"--n {args.n} --warmup {args.warmup}` from the kernel trace it leaves:\n",
         f"```\n{run_cmd}\n```\n",
         f"Mean over {len(timed) // len(LAYERS)} applications (after {args.warmup} untimed).  FLOPs count the real "
         "channels (2 x taps x cin x cout per output point; the matrix cores also multiply the zero padding of "
         "the 4-channel input and the 2-channel output); bytes are the layer's BF16 activations in and out "
         "(FP32 for the output).\n",
         "| layer | level | cin -> cout | kernel | us | GFLOP | TFLOP/s | of MFMA peak | GB | GB/s | of HBM peak |",
         "|---|---:|---|---|---:|---:|---:|---:|---:|---:|---:|"]
    tot_us = tot_f = tot_b = 0.0
    for name, lv, p, cin, cout, flops, byts in rows:
        us = sum(per[name]) / max(1, len(per[name])) / 1e3
        tot_us += us
        tot_f += flops
        tot_b += byts
        tf = flops / (us * 1e-6) / 1e12 if us > 0 else 0.0
        gbs = byts / (us * 1e-6) / 1e9 if us > 0 else 0.0
        L.append(f"| {name} | {lv} | {cin} -> {cout} | `{kname.get(name, '?')}` | {us:.1f} | {flops / 1e9:.1f} | "
                 f"{tf:.1f} | {tf / MFMA_PEAK:.3f} | {byts / 1e9:.3f} | {gbs:.0f} | {gbs / HBM_PEAK:.3f} |")
    tf = tot_f / (tot_us * 1e-6) / 1e12
    L.append(f"| all | | | | {tot_us:.1f} | {tot_f / 1e9:.1f} | {tf:.1f} | {tf / MFMA_PEAK:.3f} | "
             f"{tot_b / 1e9:.3f} | {tot_b / (tot_us * 1e-6) / 1e9:.0f} | |")
    out = os.path.join(args.out, f"net_layers_{args.dim}d_{args.nimg}x{args.n}.md")
    with open(out, "w") as fh:
        fh.write("\n".join(L) + "\n")
    print("\n".join(L))


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="mode", required=True)
    for m in ("run", "summarize"):
        s = sub.add_parser(m)
        if m == "summarize":
            s.add_argument("folder")
            s.add_argument("--out", default=os.path.join(ROOT, "profiles"))
        s.add_argument("--dim", type=int, default=2)
        s.add_argument("--nimg", type=int, default=60)
        s.add_argument("--n", type=int, default=577)
        s.add_argument("--warmup", type=int, default=2)
        s.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    run(args) if args.mode == "run" else summarize(args)


if __name__ == "__main__":
    main()
