#!/usr/bin/env python
"""Benchmark: Parareal time-to-solution on one MI355X for the Black-Scholes
network-coarse workload (European call K=100, r=0.05, sigma=0.2, T=1,
S in [0, 300]; M = 1024 interior nodes, N = 32 slices, 512 Crank-Nicolson
steps per slice, FP64 state; coarse = 4 x 64 tanh network trained on that
call, anchoring one implicit-Euler step per slice; tol 1e-8 on the max-norm
change of the iterate).

One "step" is one whole Parareal solve from the payoff to convergence.
Prints ONE JSON line.  `value` = fine cell-updates per second of the solve:
Crank-Nicolson cell updates executed by all its F sweeps divided by its
time-to-solution.  Also reported: iterations, time-to-solution, the same
solve with the numerical coarse propagator, serial fine integration on the
same GPU, the dominant kernel against its roofline, and the CPU oracle timed
on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--coarse pinn|ie]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Parareal time-to-solution & iters (PINN vs numeric G); fine cell-updates/s"
FP64_VALU_PEAK_TFLOPS = 78.6
FLOPS_PER_CELL = 10.0  # one Crank-Nicolson cell update with precomputed factors


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


# Sources of the F kernel; a traffic figure taken from counters is reported
# only while they are unchanged since the counters were taken.
F_KERNEL_SOURCES = ["bsp_propagate.hip", "bsp_steps.hpp", "bsp_tridiag.hpp",
                    "bsp_tridiag_hier.hpp", "bsp_tridiag_large.hpp", "bsp_common.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_theta_batch_pinn_call_M1024_N32_traffic.json")


def f_kernel_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in F_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2303_03848_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(shapes, M):
    """HBM bytes per F system from the committed counter summary, if it was
    taken on the current F sources with the block shape in use."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != f_kernel_hash() or t.get("M") != M:
        return None
    if shapes is None or list(shapes.get("fine") or []) != t.get("fine_shape"):
        return None
    return {"bytes_per_system": t["hbm_bytes_per_system"],
            "bytes_per_launch": t.get("hbm_bytes_per_launch", 0.0),
            "source": os.path.relpath(TRAFFIC_FILE, ROOT)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--coarse", choices=["pinn", "ie"], default="pinn")
    ap.add_argument("--train-steps", type=int, nargs=2, default=(6000, 4000),
                    metavar=("HI", "LO"), help="Adam steps at lr 1e-2 and 1e-3")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison solves")
    ap.add_argument("--fine-shape", type=int, nargs=2, metavar=("T", "MC"),
                    help="pin the F block shape (threads, nodes per thread) instead of tuning")
    ap.add_argument("--sweep-shape", type=int, nargs=2, metavar=("T", "MC"),
                    help="pin the sweep block shape instead of tuning")
    ap.add_argument("--all-workloads", action="store_true",
                    help="also measure the small call, a training step, the 512-option batch "
                         "and the 16384-node put (reported under other_workloads)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain elementwise copy of MIB MiB (float64) so a "
                         "counter profile of this command has a copy kernel of known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the "
              "slices would shard across GPUs in contiguous blocks, the serial sweep passing "
              "the boundary state from one GPU to the next)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2303_03848_amd as bsp
    from workloads import PINN_CALL, option_params

    cfg = PINN_CALL
    p = option_params(cfg)  # the benchmark workload: 1024-node call, 32 slices
    M, N, Sf, tol = cfg["M"], cfg["N"], cfg["fine_steps"], cfg["tol"]
    torch.cuda.init()
    dev = torch.device("cuda:0")
    log(f"[bench] device {torch.cuda.get_device_name(dev)}; workload {cfg['name']}")

    if args.calibrate_copy > 0:
        # Two plain copies of known size: the vectorised one (16+ bytes per
        # lane) and, through a buffer offset by one element, the scalar one
        # (8 bytes per lane, consecutive lanes on consecutive doubles: the
        # access pattern of the solver's staged loads and stores).
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.rand(n + 1, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src[:n], out=dst[:n])
        torch.cuda.synchronize()
        torch.neg(src[1:], out=dst[1:])
        torch.cuda.synchronize()
        log(f"[bench] calibration copies: {n} doubles each ({8 * n} bytes read, {8 * n} written)")
        del src, dst

    shapes = None
    if args.fine_shape or args.sweep_shape:
        if args.fine_shape:
            bsp.bs_tune_set_shape(0, M, M, *args.fine_shape)
        if args.sweep_shape:
            bsp.bs_tune_set_shape(1, M, M, *args.sweep_shape)
        shapes = {"fine": args.fine_shape, "sweep": args.sweep_shape, "source": "pinned"}
    elif not args.no_autotune:
        from paper_2303_03848_amd import autotune
        ent = autotune.tune_workload(cfg["name"], p, M, N, Sf, use_cache=False)
        shapes = {"fine": list(ent["fine"]), "sweep": list(ent["sweep"]), "source": "autotuned"}
        log(f"[bench] autotuned block shapes: fine {ent['fine']} sweep {ent['sweep']}")

    net = None
    kind = bsp.COARSE_IE
    train_info = None
    if args.coarse == "pinn":
        from paper_2303_03848_amd.pinn import train_call_network
        t0 = time.time()
        net, train_info = train_call_network(cfg, *args.train_steps)
        kind = bsp.COARSE_PINN_IE
        log(f"[bench] network trained in {time.time() - t0:.1f}s: {train_info}")

    pr = bsp.Parareal(p, M, N, Sf, 1, kind, net)

    def solve():
        return pr.solve(tol)

    for w in range(args.warmup):
        it, d, _ = solve()
        log(f"[bench] warmup {w}: iters {it}, last defect {d[-1]:.3e}")

    torch.cuda.synchronize()
    bsp.bs_profile_enable(True)
    iters_all = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        it, d, _ = solve()
        iters_all.append(it)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = bsp.bs_profile_read()
    bsp.bs_profile_enable(False)
    ms_per_step = 1e3 * elapsed / args.steps
    log(f"[bench] timed {args.steps} solves: {ms_per_step:.3f} ms each, iters {iters_all}")

    cells = prof["fine_cells"] / args.steps
    value = cells / (ms_per_step / 1e3)
    # Inside the solve the fine work of every iteration runs in one launch
    # with the sweeps (k_parareal_persist; grids up to 1024 nodes), each
    # slice waiting for its initial value, so no launch there is fine work
    # alone.  The dominant kernel's roofline is taken from the same step code
    # launched on its own: the fine launch of a full iteration (all N slices,
    # Sf steps each) on the solve's resident state, timed with events on the
    # stream it runs on.
    solve_launch_ms = prof["fine_ms"] / max(prof["fine_launches"], 1)
    u_f = pr.U[:N].contiguous()
    out_f = torch.empty_like(u_f)
    tau_f = torch.arange(N, dtype=torch.float64, device=dev) * (p["T"] / N)
    reps_f = 20
    bsp.bs_fine_propagate_batch(p, M, tau_f, p["T"] / N, Sf, u_f, out_f)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps_f):
        bsp.bs_fine_propagate_batch(p, M, tau_f, p["T"] / N, Sf, u_f, out_f)
    ev1.record()
    ev1.synchronize()
    f_ms = ev0.elapsed_time(ev1) / reps_f
    if args.calibrate_copy > 0:
        # counter runs: the same launch over fewer slices as well, so that a
        # fit separates the bytes per system from the bytes per launch
        for ns in (8, 16, 24):
            bsp.bs_fine_propagate_batch(p, M, tau_f[:ns], p["T"] / N, Sf, u_f[:ns], out_f[:ns])
        torch.cuda.synchronize()
    sys_per_launch = float(N)
    achieved = sys_per_launch * Sf * M * FLOPS_PER_CELL / (f_ms / 1e3) / 1e12
    # algorithmic HBM bytes of one F launch: each system reads its slice state
    # and writes F of it, M doubles each way
    alg_bytes = 16.0 * M * sys_per_launch
    traffic = measured_traffic(shapes, M)
    # the serial sweep on its own: the sweep launch of one synchronous
    # iteration (iteration 1: all N slices), timed with events
    pr.start()
    bsp.bs_profile_enable(True)
    pr.iterate(1)
    prof1 = bsp.bs_profile_read()
    bsp.bs_profile_enable(False)
    sweep_ms = prof1["sweep_ms"] / max(prof1["sweep_launches"], 1)
    log(f"[bench] F alone: {f_ms * 1e3:.1f} us per launch ({N} slices x {Sf} steps); "
        f"solve launches: {solve_launch_ms * 1e3:.1f} us each")

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "M": M, "N": N, "fine_steps": Sf,
                   "coarse": "pinn_ie" if kind == bsp.COARSE_PINN_IE else "implicit_euler",
                   "coarse_steps": 1, "tol": tol,
                   "network": (f"{cfg['depth']}x{cfg['width']} tanh "
                               f"{'bf16' if net is not None and net.precision else 'fp32'}"
                               if net is not None else None)},
        "iters": iters_all[-1],
        "time_to_solution_ms": ms_per_step,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                     # scaled HBM bytes per F launch: per-system bytes x systems per
                     # launch + the per-launch bytes
                     "traffic": (None if traffic is None
                                 else traffic["bytes_per_system"] * sys_per_launch
                                 + traffic["bytes_per_launch"]),
                     "kernel": "k_theta_batch (Crank-Nicolson F, all slices of one iteration)",
                     "avg_launch_ms": f_ms, "launches_timed": reps_f,
                     "systems_per_launch": sys_per_launch, "steps_per_system": Sf,
                     "flops_per_cell": FLOPS_PER_CELL,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "traffic_source": None if traffic is None else traffic["source"]},
        "block_shapes": shapes,
        "solve_launch_ms": solve_launch_ms,
        "solve_launches_per_solve": prof["fine_launches"] / args.steps,
        "sweep_alone_ms": sweep_ms,
    }
    if train_info is not None:
        out["training"] = train_info

    if not args.no_compare:
        comp = {}

        def timed_solve(pr_x, reps=3):
            pr_x.solve(tol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                it_x, d_x, _ = pr_x.solve(tol)
            torch.cuda.synchronize()
            return {"iters": it_x, "first_defect": d_x[0],
                    "time_to_solution_ms": 1e3 * (time.perf_counter() - t0) / reps}

        if kind != bsp.COARSE_IE:
            comp["numeric_coarse"] = timed_solve(bsp.Parareal(p, M, N, Sf, 1, bsp.COARSE_IE))
            net32 = bsp.PinnNet(net.params, net.n_in, net.depth, net.width, bsp.PREC_FP32)
            comp["pinn_coarse_fp32_network"] = timed_solve(
                bsp.Parareal(p, M, N, Sf, 1, bsp.COARSE_PINN_IE, net32))
            # BF16 network against the FP32 network on the Parareal grid, price units
            from paper_2303_03848_amd.pinn import grid_values
            vb = grid_values(net, p, M, N).double()
            vf = grid_values(net32, p, M, N).double()
            comp["bf16_network_max_abs_diff_vs_fp32"] = float((vb - vf).abs().max()) * p["K"]
        # serial fine integration on the same GPU: one system, N * Sf steps
        u0 = bsp.bs_initial(p, M).reshape(1, M)
        tau0 = torch.zeros(1, dtype=torch.float64, device=dev)
        bsp.bs_fine_propagate_batch(p, M, tau0, p["T"], N * Sf, u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bsp.bs_fine_propagate_batch(p, M, tau0, p["T"], N * Sf, u0)
        torch.cuda.synchronize()
        comp["serial_fine_gpu_ms"] = 1e3 * (time.perf_counter() - t0)
        # speedup bound of the paper's eq. (8) with measured per-slice costs (P = N)
        c_f = f_ms
        c_c = sweep_ms / N
        K_it = iters_all[-1]
        comp["speedup_bound_eq8"] = 1.0 / ((1 + K_it / N) * c_c / c_f + K_it / N)
        comp["speedup_vs_serial_fine"] = comp["serial_fine_gpu_ms"] / ms_per_step
        out["comparisons"] = comp

    if args.all_workloads:
        from paper_2303_03848_amd.workload_bench import measure_all
        bsp.bs_tune_reset()  # the other workloads use the default block shapes
        out["other_workloads"] = measure_all(log)

    if not args.no_cpu_baseline:
        import oracle
        threads = min(N, cpu_cores())
        po = oracle.params_from(p)
        # whole oracle solves, repeated until about 10 s of CPU time (at most 30 s)
        reps, t_all = 0, 0.0
        while t_all < 10.0 and reps < 200:
            t0 = time.perf_counter()
            r = oracle.parareal(po, M, N, Sf, 1, oracle.COARSE_IE, tol=tol, nthreads=threads)
            t_all += time.perf_counter() - t0
            reps += 1
            if t_all > 30.0:
                break
        dt = t_all / reps
        ora_cells = r["iters"] * N * Sf * M
        out["cpu_baseline"] = {
            "value": ora_cells / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": (f"{reps} oracle Parareal solves, numerical coarse, on the full "
                       f"{cfg['name']} grid ({r['iters']} iterations each, F over slices on "
                       f"{threads} threads): {t_all:.2f} s in all, {dt * 1e3:.1f} ms each"),
            "time_to_solution_ms": 1e3 * dt}
        log(f"[bench] cpu oracle: {reps} solves in {t_all:.2f}s, {r['iters']} iters, "
            f"{threads} threads")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
