"""Benchmark: batched Helmholtz solves per second at relative residual 1e-6.

Workload (default): 512 x 512 interior + 20-cell absorbing layer at 10 points
per background wavelength, refractive index 1.333 + 8 seeded Gaussian blobs,
60 plane waves in [-60, 60] degrees, all solved as one batch.  A step is one
pass of the hot path over that batch: plane-wave right-hand sides, then the
batched multigrid-preconditioned FGMRES solve to a true relative residual of
1e-6 (inputs resident on the GPU; set-up excluded and reported separately).

Printed: one JSON line with the metric, the roofline of the dominant kernel
(measured with HIP events on the library's stream in an extra profiled step)
and the FP64 CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KBH = 2 * 3.141592653589793 / 10.0  # 10 points per background wavelength
N_B = 1.333


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="blobs512x60")
    p.add_argument("--levels", type=int, default=None,
                   help="multigrid levels; default 7 in 2D (coarsest ~10^2 at 512^2), 5 in 3D (coarsest 12^3 at 128^3: "
                        "more levels would enlarge the extended grid from 177^3 to 193^3)")
    p.add_argument("--restart", type=int, default=None,
                   help="restart length m; default 10 in 2D (2.7%% faster than 8 at 512^2 x 60, 4%% at 1024^2 x 120; "
                        "basis condition ~1e5), 8 in 3D")
    p.add_argument("--cycle", type=int, default=3, help="1 = V, 2 = W, 3 = two coarse corrections on the finest "
                                                          "level and V-cycles below")
    p.add_argument("--reorth", type=int, default=0)
    p.add_argument("--krylov", choices=("sstep", "fgmres", "bicgstab"), default="sstep",
                   help="GMRES(m) in s-step form (Gram matrix + Cholesky QR), as FGMRES (Arnoldi), or the "
                        "paper's Bi-CGSTAB (restart = iterations between status checks)")
    p.add_argument("--rhs", type=int, default=None, help="override the number of plane waves")
    p.add_argument("--max-iters", type=int, default=20000, help="cap on multigrid cycles per solve")
    p.add_argument("--no-profile", action="store_true")
    p.add_argument("--no-tune", action="store_true", help="keep the default multigrid launch shapes")
    p.add_argument("--tune-cache", default=None, help="JSON-lines cache of the autotuner's choices")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="length of each bounded oracle run of the CPU baseline (one thread; one per core)")
    p.add_argument("--no-disk128-timing", action="store_true",
                   help="skip the disk128 CPU timing (set-up and solve, median of 5)")
    p.add_argument("--kappa-im", type=float, default=None,
                   help="imaginary part of the shift kappa (real part 1); default 0.4 for 2D media of contrast up to "
                        "0.1 (measured best with --omega 0.9 at 512^2 x 60), else 0.5 (strongly scattering 2D media "
                        "and 3D)")
    p.add_argument("--omega", type=float, default=None,
                   help="damped-Jacobi factor; default 0.9 with the 0.4 shift, else 0.8 (in 3D the 7-point Jacobi "
                        "smoother diverges on more modes above 6/7)")
    p.add_argument("--no-vcycle-leg", action="store_true",
                   help="skip the same workload with the paper's V-cycle (Alg. 2, CycleType 1)")
    p.add_argument("--sweep", action="store_true",
                   help="instead of the benchmark line: solves/s and cycles per solve over the shift, the cycle "
                        "type, the smoothing steps and factor, and the level count (one JSON line per setting)")
    p.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner comparison")
    p.add_argument("--learned-media", type=int, default=12, help="at most this many training media for the network")
    p.add_argument("--learned-pairs", type=int, default=20000,
                   help="training pairs the network is trained on at most: media are added until this many")
    p.add_argument("--learned-steps", type=int, default=3000, help="Adam steps of the network training")
    p.add_argument("--learned-accept", type=float, default=None,
                   help="acceptance threshold: the network's output is used where ||v - A net(v)|| <= t ||v||; "
                        "default 0.85 in 2D, 0.7 in 3D (measured: 2D 1.0 / 0.85 / 0.7 / 0.55 gave 0.97 / 0.92 / 0.94 "
                        "/ 1.00x the multigrid cycles, 3D 1.0 / 0.7 / 0.5 gave 1.26 / 0.87 / 0.94x)")
    p.add_argument("--learned-rhs", type=int, default=None,
                   help="plane waves of the learned-vs-multigrid comparison (default: all in 2D, 8 in 3D, where "
                        "one network application costs about 17 multigrid cycles); both preconditioners solve the "
                        "same sub-batch")
    p.add_argument("--no-graph", action="store_true", help="launch every kernel eagerly (for counter collection)")
    p.add_argument("--fused-step", type=int, default=2, choices=(0, 1, 2),
                   help="finest level of the s-step basis: 0 separate kernels, 1 one kernel for the up-leg, "
                        "basis matvec and next down-leg, 2 the up-leg and basis matvec in one kernel")
    p.add_argument("--copy-probe", type=float, default=256.0,
                   help="MiB of a plain device-to-device copy timed before the solve (0: skip); the same copy "
                        "calibrates the HBM byte counters")
    return p.parse_args()


def recorded_traffic(kernel, cfg):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE / WRITE_SIZE record in
    profiles/ (scaled by the copy calibration); None unless the record is for this kernel and
    launch configuration and the kernel sources are unchanged since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"traffic_{cfg['workload']}.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("config") != cfg:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def copy_probe(mib):
    """Plain device copy of `mib` MiB, three times: achievable HBM bandwidth (read + write bytes / time)."""
    import torch

    n = int(mib * 2 ** 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    return {"bytes_per_copy": 2 * 4 * n, "ms": ms, "GB/s": 2 * 4 * n / (ms * 1e-3) / 1e9}


def host_cpu():
    """(CPU model, usable host cores) of the machine running the benchmark."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def _oracle_iteration_rate(nmap, levels, restart, cycle, budget_s, theta_deg=0.0, kappa=1 + 0.5j, omega=0.8):
    """Seconds per MG-FGMRES iteration of the FP64 oracle on one right-hand side (one host thread):
    a bounded run of about budget_s seconds."""
    from threadpoolctl import threadpool_limits

    import numpy as np

    from oracle.discretization import Problem, helmholtz_matrix
    from oracle.krylov import fgmres
    from oracle.model import rhs
    from oracle.multigrid import Hierarchy

    with threadpool_limits(1):
        prob = Problem(nmap, k0h=KBH / N_B, w=20, levels=levels, beta=0.15, kappa=kappa, omega_jac=omega)
        hier = Hierarchy(prob)
        a = helmholtz_matrix(prob)
        th = np.radians(theta_deg)
        b = (prob.h ** 2 * rhs(prob, (np.sin(th), np.cos(th)))).ravel()
        ct = [2] + [1] * (levels - 2) if cycle == 3 else cycle
        pc = (lambda r: hier.cycle(r, None, 0, ct))
        t0 = time.perf_counter()
        fgmres(lambda v: a @ v, pc, b, rtol=1e-30, restart=restart, max_iters=2)
        per_iter = (time.perf_counter() - t0) / 2
        k = int(max(2, min(400, budget_s / max(per_iter, 1e-6))))
        t0 = time.perf_counter()
        _, info = fgmres(lambda v: a @ v, pc, b, rtol=1e-30, restart=restart, max_iters=k)
        el = time.perf_counter() - t0
    return el / info.iters, info.iters, el


def _rate_worker(job):
    nmap, levels, restart, cycle, budget_s, theta, kappa, omega = job
    return _oracle_iteration_rate(nmap, levels, restart, cycle, budget_s, theta, kappa, omega)


def cpu_rates(nmap, levels, restart, cycle, budget_s, kappa, omega):
    """The FP64 oracle's iteration rate on the host, before the GPU is touched (the all-cores leg
    forks worker processes): one thread on one right-hand side, and one process per usable core,
    each on its own right-hand side (angles spread over [-60, 60] degrees)."""
    import multiprocessing as mp

    model, cores = host_cpu()
    one = _oracle_iteration_rate(nmap, levels, restart, cycle, budget_s, 0.0, kappa, omega)
    thetas = [(-60.0 + 120.0 * q / max(1, cores - 1)) for q in range(cores)]
    jobs = [(nmap, levels, restart, cycle, budget_s, th, kappa, omega) for th in thetas]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_rate_worker, jobs)
    wall = time.perf_counter() - t0
    iters_all = sum(r[1] for r in res)
    return {"model": model, "cores": cores, "one_thread_s_per_iter": one[0], "one_thread_iters": one[1],
            "one_thread_s": one[2], "all_cores_iters": iters_all, "all_cores_wall_s": wall}


def cpu_baseline(rates, iters_per_solve, restart):
    """Solves/s of the FP64 oracle MG-FGMRES on all host cores (one process per core, each solving its
    own right-hand side), from bounded runs scaled by the GPU's iterations per solve."""
    per_solve_all = rates["all_cores_wall_s"] / rates["all_cores_iters"] * iters_per_solve
    one = 1.0 / (rates["one_thread_s_per_iter"] * iters_per_solve)
    return {
        "value": 1.0 / per_solve_all,
        "unit": "solves/s",
        "cores": rates["cores"],
        "kind": "oracle",
        "cpu_model": rates["model"],
        "one_thread_value": one,
        "sample": (f"FP64 oracle MG-FGMRES({restart}), one process per core on {rates['cores']} cores "
                   f"({rates['model']}), each on its own right-hand side: {rates['all_cores_iters']} iterations "
                   f"in {rates['all_cores_wall_s']:.1f} s wall; one thread alone: {rates['one_thread_iters']} "
                   f"iterations in {rates['one_thread_s']:.1f} s; scaled by {iters_per_solve:.0f} iterations per "
                   f"solve (the GPU's mean at the same parameters); set-up excluded"),
    }


def cpu_disk128_timing(reps=5):
    """The small CPU configuration (disk128: 128^2 interior, 20-cell layer, disk of radius 20 cells and
    contrast 0.05, one normal-incidence plane wave, complex128 MG-FGMRES(20), 4 levels, rel. residual
    1e-6): set-up and solve timed separately, median of `reps` after a warm-up, with one BLAS thread
    (the paper's one-thread protocol, Sec. VI) and with all usable cores."""
    from threadpoolctl import threadpool_limits

    import numpy as np

    import synth
    from oracle.discretization import Problem, helmholtz_matrix
    from oracle.krylov import fgmres
    from oracle.model import rhs
    from oracle.multigrid import Hierarchy

    model, cores = host_cpu()
    nmap = synth.workload_medium("disk128")
    out = {"workload": "disk128", "cpu_model": model, "repetitions": reps}
    for label, nth in (("one_thread", 1), ("all_cores", cores)):
        with threadpool_limits(nth):
            ts, tv, its = [], [], []
            for rep in range(reps + 1):
                t0 = time.perf_counter()
                prob = Problem(nmap, k0h=KBH / N_B, w=20, levels=4, beta=0.15)
                hier = Hierarchy(prob)
                a = helmholtz_matrix(prob)
                b = (prob.h ** 2 * rhs(prob, (0.0, 1.0))).ravel()
                t1 = time.perf_counter()
                _, info = fgmres(lambda v: a @ v, hier.vcycle, b, rtol=1e-6, restart=20, max_iters=2000)
                t2 = time.perf_counter()
                if rep:  # the first pass warms up
                    ts.append(t1 - t0)
                    tv.append(t2 - t1)
                    its.append(info.iters)
        out[label] = {"threads": nth, "setup_s_median": float(np.median(ts)), "solve_s_median": float(np.median(tv)),
                      "iterations": int(its[-1]), "converged": bool(info.converged),
                      "rel_res_true": float(info.rel_res_true)}
    return out


def gradient_leg(ctx, dirs, nmap, reps=3):
    """One data-term gradient evaluation of the inverse problem (Sec. V, Prop. 1) with on-grid
    receivers on the transmission-side row: forward solves of all plane waves, data residual,
    adjoint solves, grad_f.  Data: the forward field of a medium with half the contrast, so
    that the residual is not trivial.  Reported: mean wall time over `reps` evaluations."""
    import numpy as np
    import torch

    from paper_2107_03679_amd.autograd import receiver_line

    dev = torch.device("cuda:0")
    rx = receiver_line(ctx)
    half = 1.333 + 0.5 * (nmap - 1.333)
    ctx.update_n(torch.tensor(half, dtype=torch.float32, device=dev))
    u, _ = ctx.solve(ctx.plane_wave_rhs(dirs))
    y = ctx.sample(rx, u)
    ctx.update_n(torch.tensor(nmap, dtype=torch.float32, device=dev))
    rhs, uin = ctx.plane_wave_rhs(dirs, with_uin=True)

    def once():
        usc, st = ctx.solve(rhs)
        res, loss = ctx.data_residual(rx, usc, y)
        lam, st_a = ctx.adjoint(ctx.sample_adjoint(rx, res))
        g = ctx.grad_f(usc, lam, u_in=uin)
        return st, st_a, loss, g

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st, st_a, loss, g = once()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    return {"ms_per_gradient": 1e3 * el, "forward_iters_mean": float(st.iters.mean()),
            "adjoint_iters_mean": float(st_a.iters.mean()), "converged": bool(st.converged and st_a.converged),
            "loss": loss, "receivers": int(rx.numel()), "plane_waves": int(dirs.shape[0])}


def progress(msg):
    """A progress line on stderr (the benchmark line itself is the only stdout output)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def learned_leg(make_ctx, args, wl, nmap, dirs, mg_iters_mean, mg_value):
    """Learned-FGMRES on the same workload: the network is trained on the GPU on residual/error
    pairs from MG-FGMRES solves of training media (blob seeds 1000 + i, random angles), then
    used as z = net(v) + V(v - A net(v)) with the acceptance test and V-cycle fallback."""
    import numpy as np
    import torch

    import synth
    from paper_2107_03679_amd import learned

    dev = torch.device("cuda:0")
    kind, kw = wl["medium"]
    B = dirs.shape[0]
    d = wl["d"]
    # large crops: the U-Net's coarsest level has to see a good part of the grid, as it does in the solver
    crop = 256 if d == 2 else 96
    # a context of its own, capped at 3x the multigrid cycles per solve
    ctx = make_ctx(args.cycle, max_iters=int(3 * mg_iters_mean) + 16)
    Bl = args.learned_rhs or (B if d == 2 else min(B, 8))
    sub = np.round(np.linspace(0, B - 1, Bl)).astype(int)
    ldirs = dirs[sub]
    rng = np.random.default_rng(5)
    t0 = time.perf_counter()
    sets = []
    n_train, i = 0, 0
    while True:  # training media until the pair budget (or the media count) is reached, then one to validate
        val_medium = n_train >= args.learned_pairs or i == args.learned_media
        m = synth.blob_map(wl["n"], kw["n_blobs"], kw["sigma_range"], kw["amp_hi"], 1000 + i,
                           max_dn=kw.get("max_dn"), d=d)
        ctx.update_n(torch.tensor(m, dtype=torch.float32, device=dev))
        if d == 2:
            th = np.radians(rng.uniform(-60.0, 60.0, B))
            train_dirs = np.stack([np.sin(th), np.cos(th)], 1)
        else:  # the 45-degree cone at random azimuths
            ph = rng.uniform(0.0, 2 * np.pi, B)
            a = np.radians(45.0)
            train_dirs = np.stack([np.sin(a) * np.cos(ph), np.sin(a) * np.sin(ph), np.full(B, np.cos(a))], 1)
        rhs = ctx.plane_wave_rhs(train_dirs)
        progress(f"learned: {'validation' if val_medium else 'training'} pairs from medium {i}")
        # 3D: one 96^3 crop per snapshot and right-hand side (each is 21 MB of FP32 features and targets)
        sets.append(learned.collect(ctx, [rhs], size=crop, crops_per_snapshot=1 if (val_medium or d == 3) else 4,
                                    every_cycles=8 if d == 2 else 4, max_snaps=12 if d == 2 else 4, seed=1000 + i,
                                    out=None if (val_medium or not sets) else sets.pop()))
        if val_medium:
            break
        n_train = sets[-1].feat.shape[0]
        i += 1
    n_media = i
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    ctx.update_n(torch.tensor(nmap, dtype=torch.float32, device=dev))
    tr, val = sets
    val = learned.rescaled(ctx, val, tr.gamma)
    progress(f"learned: training on {tr.feat.shape[0]} pairs")
    net = learned.new_network(11, dim=d)
    log = learned.train(net, tr, steps=args.learned_steps, batch=4 if d == 2 else 2, lr=1e-4, seed=3,
                        err_weight=0.0, res_weight=1.0)
    ratio = learned.residual_ratio(ctx, net, val)
    # the multigrid baseline on the same plane waves, same context (s-step GMRES, autotuned shapes)
    x = ctx.empty_fields(Bl)
    ctx.autotune(Bl)
    ctx.solve(ctx.plane_wave_rhs(ldirs), out=x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st_mg = ctx.solve(ctx.plane_wave_rhs(ldirs), out=x)
    torch.cuda.synchronize()
    mg_sub = Bl / (time.perf_counter() - t0)
    progress(f"learned: {Bl} solves with the network")
    ctx.set_preconditioner(net, accept_tol=args.learned_accept, gamma=tr.gamma, mode="then_mg")
    # profiled warm-up solve: the network's MFMA rate
    ctx.profile(True)
    ctx.solve(ctx.plane_wave_rhs(ldirs), out=x)
    rep = ctx.profile_report()
    ctx.profile(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = ctx.solve(ctx.plane_wave_rhs(ldirs), out=x)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.set_preconditioner(None)
    ne = ctx.info.n_e
    ctx.close()
    net_ms, net_launches, _ = rep.get("net_apply", (0.0, 0, 0.0))
    fl = (learned.flops_per_image(ne, ne) if d == 2 else learned.flops_per_image(ne, ne, ne)) * Bl
    achieved = fl * net_launches / (net_ms * 1e-3) / 1e12 if net_ms > 0 else 0.0
    net.close()
    value = Bl / el
    return {
        "value": value, "unit": "solves/s", "rhs": Bl, "multigrid_same_rhs": mg_sub, "vs_multigrid": value / mg_sub,
        "iters_mean": float(st.iters.mean()), "iters_max": int(st.iters.max()),
        "multigrid_iters_mean": float(st_mg.iters.mean()),
        "iters_vs_multigrid": float(st.iters.mean()) / float(st_mg.iters.mean()),
        "all_converged": bool(st.converged), "rel_res_true_max": float(st.rel_res_true.max()),
        "accepted_frac": float(1.0 - st.fallbacks.sum() / max(1, st.iters.sum())),
        "pairs": int(tr.feat.shape[0]), "crop": crop, "train_steps": log.steps, "train_s": log.seconds,
        "collect_s": t_collect, "heldout_residual_ratio": ratio, "training_media": n_media,
        "mode": f"z = net(v) + V-cycle(v - A net(v)), V-cycle alone where ||v - A net(v)|| > "
                f"{args.learned_accept:g} ||v||",
        "mfma": {"kernel": "net_apply (all convolutions of one application)", "achieved": achieved,
                 "peak": 2500.0, "unit": "TFLOP/s", "frac": achieved / 2500.0, "flops_per_launch": fl,
                 "ms_per_launch": net_ms / max(1, net_launches)},
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; the batch of plane waves is the data-parallel "
                                   "axis and multi-GPU runs are not part of it", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np

    import synth

    wl = synth.WORKLOADS[args.workload]
    kind, mp = wl["medium"]
    weak = wl["d"] == 2 and mp.get("amp_hi", mp.get("dn", 0.0)) <= 0.1  # 2D, contrast up to 0.1
    if args.kappa_im is None:
        args.kappa_im = 0.4 if weak else 0.5
    if args.omega is None:
        args.omega = 0.9 if weak else 0.8
    if args.levels is None:
        args.levels = 7 if wl["d"] == 2 else 5
    if args.restart is None:
        args.restart = 10 if wl["d"] == 2 else 8
    if args.learned_accept is None:
        args.learned_accept = 0.85 if wl["d"] == 2 else 0.7
    nmap = synth.workload_medium(args.workload).astype(np.float32).astype(np.float64)
    dirs = synth.workload_directions(args.workload, args.rhs)
    B = dirs.shape[0]
    if args.sweep:
        return sweep(args, wl, nmap, dirs)
    # host legs first: the all-cores leg forks worker processes, which must happen before the GPU is used
    rates = disk = None
    if not args.no_cpu_baseline and wl["d"] == 2:
        progress("CPU oracle rates (one thread; one process per core)")
        rates = cpu_rates(nmap, args.levels, args.restart, args.cycle, args.cpu_seconds, complex(1.0, args.kappa_im),
                          args.omega)
        if not args.no_disk128_timing:
            progress("CPU oracle, disk128 set-up and solve timing")
            disk = cpu_disk128_timing()
    import torch

    from paper_2107_03679_amd import helm

    w = 20
    ne = helm.extended_size(wl["n"], w, args.levels)
    k0 = (KBH / N_B) * (ne - 1)
    dev = torch.device("cuda:0")

    def make_ctx(cycle, max_iters=None):
        return helm.Context(torch.tensor(nmap, dtype=torch.float32, device=dev), k0, abl_width=w, beta=wl["beta"],
                            levels=args.levels, restart=args.restart, cycle=cycle, reorth=args.reorth, max_batch=B,
                            max_iters=args.max_iters if max_iters is None else max_iters, use_graph=0 if args.no_graph else 1, fused_step=args.fused_step,
                            kappa=complex(1.0, args.kappa_im), omega_jac=args.omega,
                            krylov={"sstep": helm.KRYLOV_SSTEP, "fgmres": helm.KRYLOV_FGMRES,
                                    "bicgstab": helm.KRYLOV_BICGSTAB}[args.krylov])

    progress("GPU set-up")
    t_setup = time.perf_counter()
    ctx = make_ctx(args.cycle)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    tune = None
    if not args.no_tune:
        t_tune = time.perf_counter()
        tune = ctx.autotune(B, cache=args.tune_cache)
        tune["tune_s"] = time.perf_counter() - t_tune
    x = ctx.empty_fields(B)
    probe = copy_probe(args.copy_probe) if args.copy_probe > 0 else None

    def step():
        rhs = ctx.plane_wave_rhs(dirs)
        _, st = ctx.solve(rhs, out=x)
        return st

    progress(f"{args.warmup} warm-up and {args.steps} timed steps")
    for _ in range(args.warmup):
        st = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        stats.append(step())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = stats[-1]
    iters = np.concatenate([s.iters for s in stats])
    value = B * args.steps / el

    out = {
        "metric": "Helmholtz solves/s at rel. residual 1e-6 (512\u00b2, 60 RHS); learned vs MG-GMRES"
        if args.workload == "blobs512x60"
        else f"Helmholtz solves/s at rel. residual 1e-6 ({args.workload})",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "interior": wl["n"], "grid": ne, "rhs": B, "levels": args.levels,
            "coarsest": ctx.info.coarsest_n, "restart": args.restart, "cycle": {1: "V", 2: "W", 3: "W at the finest level, V below"}[args.cycle],
            "kappa": f"1+{args.kappa_im:g}j", "nu": [1, 1], "omega_jac": args.omega, "rtol": 1e-6,
            "preconditioner": "multigrid",
            "krylov": {"sstep": f"GMRES({args.restart}), s-step form (Gram + Cholesky QR)",
                       "fgmres": f"FGMRES({args.restart})" + (", CGS2" if args.reorth else ", CGS1"),
                       "bicgstab": "Bi-CGSTAB (Alg. 3)"}[args.krylov],
            "launch_shapes": "default" if tune is None else {
                "down_tiles": tune["down_tiles"], "up_tiles": tune["up_tiles"],
                "coarse_single_launch_max_points": tune["coarse_single_launch_max_points"],
                "up_mv_rows": tune["up_mv_rows"], "up_mv_rhs_per_block": tune["up_mv_rhs_per_block"]},
        },
        "solver": {
            "all_converged": bool(all(s.converged for s in stats)),
            "iters_mean": float(iters.mean()), "iters_max": int(iters.max()),
            "rel_res_true_max": float(max(s.rel_res_true.max() for s in stats)),
            "setup_s": t_setup,
        },
        "autotune": None if tune is None else {
            k: tune[k] for k in ("from_cache", "vcycle_ms", "vcycle_default_ms", "tune_s")},
    }

    if not args.no_profile:
        progress("profiled step")
        ctx.profile(True)
        step()
        rep = ctx.profile_report()
        ctx.profile(False)
        total = sum(v[0] for v in rep.values())
        name, (ms, n, by) = max(rep.items(), key=lambda kv: kv[1][0])
        achieved = by / (ms * 1e-3) / 1e9
        cfg = {"workload": args.workload, "rhs": B, "levels": args.levels, "restart": args.restart,
               "cycle": args.cycle, "krylov": args.krylov, "fused_step": args.fused_step}
        traffic = recorded_traffic(name, cfg)
        out["roofline"] = {
            "bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_GBs": None if traffic is None else traffic * n / (ms * 1e-3) / 1e9,
            "avg_launch_us": 1000.0 * ms / n, "bytes_per_launch": by / n, "share_of_step": ms / total,
            "record_key": cfg,
        }
        if probe is not None:
            out["roofline"]["copy_probe"] = probe
        out["kernels"] = {
            k: {"ms": round(v[0], 3), "launches": v[1], "GB/s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else 0}
            for k, v in sorted(rep.items(), key=lambda kv: -kv[1][0])
        }
    # the per-evaluation view of the inverse problem: a new medium (helm_update_n) before every batch
    t_upd = []
    nmap_t = torch.tensor(nmap, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, min(args.steps, 5))):
        t1 = time.perf_counter()
        ctx.update_n(nmap_t)
        torch.cuda.synchronize()
        t_upd.append(time.perf_counter() - t1)
        st_u = step()
    torch.cuda.synchronize()
    el_u = (time.perf_counter() - t0) / len(t_upd)
    out["with_update_n"] = {"value": B / el_u, "unit": "solves/s", "update_n_ms": 1e3 * float(np.median(t_upd)),
                            "all_converged": bool(st_u.converged),
                            "note": "helm_update_n (medium set-up on the GPU, coarsest inverse on the host) + "
                                    "right-hand sides + batched solve, per step"}
    if args.workload == "inverse256x32":
        out["gradient"] = gradient_leg(ctx, dirs, nmap)
    if not args.no_learned:
        progress("learned-preconditioner leg")
        out["learned"] = learned_leg(make_ctx, args, wl, nmap, dirs, float(iters.mean()), value)
    ctx.close()
    if not args.no_vcycle_leg and args.cycle != 1:
        progress("V-cycle leg")
        # the paper's cycle (Alg. 2, CycleType 1: one V-cycle per preconditioner application)
        vctx = make_ctx(1)
        if not args.no_tune:
            vctx.autotune(B, cache=args.tune_cache)
        xv = vctx.empty_fields(B)
        vctx.solve(vctx.plane_wave_rhs(dirs), out=xv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, min(args.steps, 5))):
            _, st_v = vctx.solve(vctx.plane_wave_rhs(dirs), out=xv)
        torch.cuda.synchronize()
        el_v = (time.perf_counter() - t0) / max(1, min(args.steps, 5))
        out["vcycle"] = {"value": B / el_v, "unit": "solves/s", "iters_mean": float(st_v.iters.mean()),
                         "iters_max": int(st_v.iters.max()), "all_converged": bool(st_v.converged),
                         "rel_res_true_max": float(st_v.rel_res_true.max())}
        vctx.close()
    if rates is not None:
        out["cpu_baseline"] = cpu_baseline(rates, float(iters.mean()), args.restart)
    if disk is not None:
        out["cpu_disk128"] = disk
    print(json.dumps(out), flush=True)


def sweep(args, wl, nmap, dirs):
    """Solves/s, cycles per solve and the certified residual over the preconditioner's settings on one
    workload (same batch, autotuned shapes per setting); one JSON line per setting."""
    import numpy as np
    import torch

    from paper_2107_03679_amd import helm

    B = dirs.shape[0]
    grid = [dict(kim=k) for k in (0.2, 0.3, 0.35, 0.4, 0.5, 0.6, 0.7)]
    grid += [dict(kim=k, om=o) for k in (0.3, 0.35, 0.4) for o in (0.85, 0.9, 0.95)]
    grid += [dict(cycle=c, kim=k) for c in (1, 2) for k in (0.35, 0.5)]
    grid += [dict(nu=2, kim=k) for k in (0.35, 0.5)]
    grid += [dict(levels=L, kim=k) for L in (5, 6) for k in (0.35, 0.5)]
    for g in grid:
        L, cyc, nu = g.get("levels", args.levels), g.get("cycle", args.cycle), g.get("nu", 1)
        ne = helm.extended_size(wl["n"], 20, L)
        k0 = (KBH / N_B) * (ne - 1)
        ctx = helm.Context(torch.tensor(nmap, dtype=torch.float32, device="cuda:0"), k0, abl_width=20,
                           beta=wl["beta"], levels=L, restart=args.restart, cycle=cyc, max_batch=B,
                           max_iters=args.max_iters, kappa=complex(1.0, g["kim"]), omega_jac=g.get("om", 0.8),
                           nu1=nu, nu2=nu)
        ctx.autotune(B)
        x = ctx.empty_fields(B)
        ctx.solve(ctx.plane_wave_rhs(dirs), out=x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = ctx.solve(ctx.plane_wave_rhs(dirs), out=x)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.close()
        print(json.dumps({"workload": args.workload, "levels": L, "cycle": cyc, "nu": nu, "kappa": [1.0, g["kim"]],
                          "omega_jac": g.get("om", 0.8), "restart": args.restart, "solves_per_s": B / el,
                          "iters_mean": float(st.iters.mean()), "iters_max": int(st.iters.max()),
                          "all_converged": bool(st.converged), "rel_res_true_max": float(st.rel_res_true.max())}),
              flush=True)


if __name__ == "__main__":
    main()
