#!/usr/bin/env python
"""Benchmark: Parareal time-to-solution on one MI355X for the Black-Scholes
equation (Parareal, Sec. 3.1 eq. (7); Crank-Nicolson fine propagator and
implicit-Euler / network coarse propagators, Secs. 3.2-3.3).

Headline workload (default, ``--workload large_put``): the largest
single-GPU configuration, a European put K=100, r=0.03, sigma=0.35, T=2,
S in [0, 400]; M = 16384 interior nodes, N = 256 slices, 2048 Crank-Nicolson
steps per slice (FP64 state), coarse = a 6 x 256 tanh network trained on that
put (FP32 training with the hand-written residual gradient, outside the timed
region) evaluated in BF16 on the matrix cores and anchoring one
implicit-Euler step per slice; tol 1e-10 on the max-norm change of the
iterate.  ``--workload pinn_call`` runs the 1024-node call (32 slices, 512
steps, 4 x 64 network, tol 1e-8) as the headline instead; by default it is
reported as a secondary entry.

One "step" is one whole Parareal solve from the payoff to convergence.
Prints ONE JSON line.  `value` = fine cell-updates per second of the solve
(Crank-Nicolson cell updates executed by all its fine launches divided by its
time-to-solution).  Also reported: iterations, the same solve with the
numerical coarse propagator, serial fine integration on the same GPU, the
dominant kernel against its roofline (timed inside the measured solves), the
CPU oracle timed on this host, and the network's error.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large_put|pinn_call]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# Sources of the large-grid F kernel; a traffic figure taken from counters is
# reported only while they are unchanged since the counters were taken.
F_SOURCES = ["bsp_propagate.hip", "bsp_steps.hpp", "bsp_tridiag.hpp", "bsp_tridiag_rc.hpp",
             "bsp_tridiag_large.hpp", "bsp_common.hpp"]


def f_kernel_hash() -> str:
    h = hashlib.sha256()
    for f in F_SOURCES:
        with open(os.path.join(ROOT, "paper_2303_03848_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path: str, workload: str):
    """HBM bytes per F launch from a committed counter summary, if it was
    taken on the current F sources for this workload."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != f_kernel_hash() or t.get("workload") != workload:
        return None
    return t


def grid_inputs(p: dict, M: int, N: int):
    """Network inputs (tau_n, S_j / K) of the Parareal grid, [(N+1) M, 2] float32."""
    import numpy as np
    import torch
    S = (np.arange(1, M + 1) * (p["s_max"] / (M + 1))) / p["K"]
    taus = np.arange(N + 1) * (p["T"] / N)
    T, X = np.meshgrid(taus, S, indexing="ij")
    return torch.tensor(np.stack([T.ravel(), X.ravel()], 1), dtype=torch.float32, device="cuda")


def network_error(bsp, net, p, M, N, U_ref):
    """Max |K v(tau_n, S_j/K) - U_ref[n, j]| over levels n >= 1 (price units)
    and the same with the network evaluated in FP32."""
    X = grid_inputs(p, M, N)
    out = {}
    for name, prec in (("bf16", bsp.PREC_BF16), ("fp32", bsp.PREC_FP32)):
        n2 = bsp.PinnNet(net.params, net.n_in, net.depth, net.width, prec)
        v = bsp.pinn_forward(n2, X).double().reshape(N + 1, M) * p["K"]
        out[name] = float((v[1:] - U_ref[1:]).abs().max())
    return out


def timed_solves(bsp, torch, pr, tol, reps):
    pr.solve(tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        it, d, _ = pr.solve(tol)
    torch.cuda.synchronize()
    return {"iters": it, "first_defect": d[0], "last_defect": d[-1],
            "time_to_solution_ms": 1e3 * (time.perf_counter() - t0) / reps}


def serial_fine_gpu_ms(bsp, torch, p, M, N, Sf):
    """Serial fine integration on the same GPU: one system, N*Sf steps."""
    u0 = bsp.bs_initial(p, M).reshape(1, M)
    tau0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    bsp.bs_fine_propagate_batch(p, M, tau0, p["T"] / N, Sf, u0)  # warm-up: one slice
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bsp.bs_fine_propagate_batch(p, M, tau0, p["T"], N * Sf, u0)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0)


def solve_and_profile(bsp, torch, pr, tol, warmup, steps):
    for w in range(warmup):
        it, d, _ = pr.solve(tol)
        log(f"[bench] warmup {w}: iters {it}, last defect {d[-1]:.3e}")
    torch.cuda.synchronize()
    bsp.bs_profile_enable(True)
    iters_all = []
    t0 = time.perf_counter()
    for _ in range(steps):
        it, d, _ = pr.solve(tol)
        iters_all.append(it)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = bsp.bs_profile_read()
    bsp.bs_profile_enable(False)
    return 1e3 * elapsed / steps, iters_all, d, prof


def bench_large_put(args, bsp, torch):
    from workloads import LARGE_PUT, option_params
    from paper_2303_03848_amd.pinn import train

    cfg = LARGE_PUT
    p = option_params(cfg)
    M, N, Sf, tol = cfg["M"], cfg["N"], cfg["fine_steps"], cfg["tol"]
    log(f"[bench] workload {cfg['name']}")
    t0 = time.time()
    net, info = train(p, cfg["n_in"], cfg["depth"], cfg["width"], bsp.PREC_FP32,
                      epochs_hi=args.large_train_epochs[0], epochs_lo=args.large_train_epochs[1])
    net.precision = bsp.PREC_BF16
    info = {k: v for k, v in info.items() if k != "history"}
    log(f"[bench] 6x256 network trained in {time.time() - t0:.1f}s: {info}")

    pr = bsp.Parareal(p, M, N, Sf, 1, bsp.COARSE_PINN_IE, net)
    ms, iters_all, defects, prof = solve_and_profile(bsp, torch, pr, tol, args.warmup, args.steps)
    log(f"[bench] timed {args.steps} solves: {ms:.3f} ms each, iters {iters_all}; F {prof}")
    cells = (prof["fine_cells"] + prof["solve_cells"]) / args.steps
    value = cells / (ms / 1e3)
    # The dominant kernel: the one-launch part of each timed solve
    # (k_large_persist: the coarse prediction and every sweep on one block,
    # the fine work of slices 1..N-1 in every iteration on the others),
    # timed with events on the stream it runs on; its algorithmic work is
    # the fine cell updates of those slices.  Slice 0's first fine
    # propagation (k_rc_theta, one system, on a side stream beside the
    # network grid) is reported beside it.
    s_ms, s_launches, s_cells = prof["solve_ms"], prof["solve_launches"], prof["solve_cells"]
    achieved = FLOPS_PER_CELL * s_cells / (s_ms / 1e3) / 1e12
    f1 = {"kernel": "k_rc_theta", "avg_launch_ms": prof["fine_ms"] / max(prof["fine_launches"], 1),
          "tflops": FLOPS_PER_CELL * prof["fine_cells"] / (prof["fine_ms"] / 1e3) / 1e12,
          "systems_per_launch": prof["fine_cells"] / (max(prof["fine_launches"], 1) * Sf * M)}
    traffic = measured_traffic(os.path.join(ROOT, "profiles", "k_large_persist_traffic.json"),
                               cfg["name"])
    U = pr.U.clone()
    # per-slice costs for eq. (8): one iteration launch after launch
    pr.start()
    bsp.bs_profile_enable(True)
    pr.iterate(1)
    p1 = bsp.bs_profile_read()
    bsp.bs_profile_enable(False)
    c_f = p1["fine_ms"] / max(p1["fine_launches"], 1)
    c_c = p1["sweep_ms"] / max(p1["sweep_launches"], 1) / N
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "M": M, "N": N, "fine_steps": Sf,
                   "coarse": "pinn_ie", "coarse_steps": 1, "tol": tol,
                   "network": f"{cfg['depth']}x{cfg['width']} tanh bf16"},
        "iters": iters_all[-1],
        "time_to_solution_ms": ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                     "traffic": None if traffic is None else traffic["hbm_bytes_per_launch"],
                     "kernel": "k_large_persist (the prediction and every sweep on one block, "
                               "the fine work of slices 1..N-1 in every iteration on one "
                               "block per slice beside it)",
                     "avg_launch_ms": s_ms / s_launches, "launches_timed": s_launches,
                     "fine_cells_per_launch": s_cells / s_launches,
                     "flops_per_cell": FLOPS_PER_CELL,
                     "algorithmic_bytes_per_launch":
                         (s_cells / s_launches) / (Sf * M) * 16.0 * M,
                     "traffic_source": None if traffic is None else
                     "profiles/k_large_persist_traffic.json"},
        "slice0_first_fine_launch": f1,
        "per_slice_costs_ms": {"c_f_fine_launch": c_f, "c_c_sweep_per_slice": c_c},
        "training": info,
        "defects": defects,
    }
    if not args.no_compare:
        comp = {}
        comp["numeric_coarse"] = timed_solves(bsp, torch, bsp.Parareal(p, M, N, Sf, 1,
                                                                         bsp.COARSE_IE), tol, 2)
        comp["pinn_coarse"] = {"iters": iters_all[-1], "time_to_solution_ms": ms,
                               "first_defect": defects[0]}
        # network error against the converged solution (the serial fine
        # solution to within tol), price units
        comp["network_max_error_vs_fine"] = network_error(bsp, net, p, M, N, U)
        comp["serial_fine_gpu_ms"] = serial_fine_gpu_ms(bsp, torch, p, M, N, Sf)
        comp["speedup_vs_serial_fine"] = comp["serial_fine_gpu_ms"] / ms
        comp["speedup_numeric_vs_serial_fine"] = (comp["serial_fine_gpu_ms"] /
                                                  comp["numeric_coarse"]["time_to_solution_ms"])
        # eq. (8) with measured per-slice costs (P = N): c_f one fine launch
        # over all slices, c_c the sweep's time per slice (launch after launch)
        K_it = iters_all[-1]
        comp["speedup_bound_eq8"] = 1.0 / ((1 + K_it / N) * c_c / c_f + K_it / N)
        out["comparisons"] = comp
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_fine(p, M, N, Sf, cfg["name"])
    return out


def cpu_baseline_fine(p, M, N, Sf, name):
    """The oracle's fine propagator (textbook Thomas, FP64) on this host: F
    over `threads` slices at once, one slice per thread, repeated for about
    10 s.  Cell-updates per second."""
    import numpy as np
    import oracle
    threads = min(N, cpu_cores())
    po = oracle.params_from(p)
    u0 = oracle.initial(po, M)
    dT = p["T"] / N

    def one(n):
        return oracle.fine(po, M, n * dT, dT, Sf, u0)

    reps, t_all, rounds = 0, 0.0, []
    with ThreadPoolExecutor(threads) as ex:
        while t_all < 10.0 and reps < 50:
            t0 = time.perf_counter()
            list(ex.map(one, range(threads)))
            rounds.append(time.perf_counter() - t0)
            t_all += rounds[-1]
            reps += 1
    # one slice on one core (serial fine integration is N of these in a row)
    t0 = time.perf_counter()
    one(0)
    t_one = time.perf_counter() - t0
    cells = reps * threads * Sf * M
    log(f"[bench] cpu oracle: {reps} rounds of {threads} slices in {t_all:.2f}s; "
        f"one slice on one core {t_one:.3f}s")
    return {"value": cells / t_all, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": (f"oracle fine propagator ({Sf} Crank-Nicolson steps on {M} nodes, the "
                       f"{name} slice) on {threads} slices at once, one per thread, {reps} "
                       f"rounds: {t_all:.2f} s; {1e3 * t_all / reps:.1f} ms per round"),
            "cpu_model": cpu_model(),
            "seconds_per_slice_round": t_all / reps,
            "seconds_per_round_std": float(np.std(rounds)),
            "one_core_seconds_per_slice": t_one,
            "one_core_serial_fine_seconds_estimate": N * t_one,
            "note": "built -O2 -ffp-contract=off (the parity build); a whole oracle Parareal "
                    "solve of this workload would take minutes"}


def bench_pinn_call(args, bsp, torch, headline: bool):
    from workloads import PINN_CALL, option_params
    from paper_2303_03848_amd.pinn import train_call_network

    cfg = PINN_CALL
    p = option_params(cfg)
    M, N, Sf, tol = cfg["M"], cfg["N"], cfg["fine_steps"], cfg["tol"]
    log(f"[bench] workload {cfg['name']}")
    t0 = time.time()
    net, info = train_call_network(cfg, *args.train_epochs)
    log(f"[bench] 4x64 network trained in {time.time() - t0:.1f}s: {info}")
    pr = bsp.Parareal(p, M, N, Sf, 1, bsp.COARSE_PINN_IE, net)
    steps = args.steps if headline else 5
    warm = args.warmup if headline else 2
    ms, iters_all, defects, prof = solve_and_profile(bsp, torch, pr, tol, warm, steps)
    cells = (prof["fine_cells"] + prof["solve_cells"]) / steps
    U = pr.U.clone()
    out = {"workload": cfg["name"], "M": M, "N": N, "fine_steps": Sf, "tol": tol,
           "coarse": "pinn_ie", "network": f"{cfg['depth']}x{cfg['width']} tanh bf16",
           "iters": iters_all[-1], "time_to_solution_ms": ms,
           "cell_updates_per_s": cells / (ms / 1e3), "training": info,
           "solve_launch_ms": prof["solve_ms"] / max(prof["solve_launches"], 1)}
    comp = {}
    comp["numeric_coarse"] = timed_solves(bsp, torch, bsp.Parareal(p, M, N, Sf, 1, bsp.COARSE_IE),
                                          tol, 5)
    net32 = bsp.PinnNet(net.params, net.n_in, net.depth, net.width, bsp.PREC_FP32)
    comp["pinn_coarse_fp32_network"] = timed_solves(
        bsp, torch, bsp.Parareal(p, M, N, Sf, 1, bsp.COARSE_PINN_IE, net32), tol, 5)
    comp["pinn_coarse_bf16_network"] = {"iters": iters_all[-1], "time_to_solution_ms": ms,
                                        "first_defect": defects[0]}
    comp["network_max_error_vs_fine"] = network_error(bsp, net, p, M, N, U)
    comp["serial_fine_gpu_ms"] = serial_fine_gpu_ms(bsp, torch, p, M, N, Sf)
    out["comparisons"] = comp
    if headline:
        out = {
            "metric": METRIC, "value": out["cell_updates_per_s"], "unit": "cell-updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": cfg["name"], "M": M, "N": N, "fine_steps": Sf,
                       "coarse": "pinn_ie", "coarse_steps": 1, "tol": tol,
                       "network": f"{cfg['depth']}x{cfg['width']} tanh bf16"},
            "iters": iters_all[-1], "time_to_solution_ms": ms, **{k: out[k] for k in
                                                                   ("training", "comparisons")},
        }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["large_put", "pinn_call"], default="large_put")
    ap.add_argument("--large-train-epochs", type=int, nargs=2, default=(190, 60),
                    metavar=("HI", "LO"),
                    help="Adam epochs (8 minibatches each) at lr 1e-2 and 1e-3 for the 6 x 256 "
                         "network")
    ap.add_argument("--train-epochs", type=int, nargs=2, default=(5000, 800),
                    metavar=("HI", "LO"),
                    help="Adam epochs at lr 1e-2 and 1e-3 for the 4 x 64 call network")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison solves")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary workload entry")
    ap.add_argument("--all-workloads", action="store_true",
                    help="also measure the small call, a training step, the 512-option batch "
                         "(reported under other_workloads)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain elementwise copy of MIB MiB (float64) so a "
                         "counter profile of this command has a copy kernel of known size")
    ap.add_argument("--calibrate-only", action="store_true",
                    help="exit after the calibration copy")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the "
              "slices would shard across GPUs in contiguous blocks, the serial sweep passing "
              "the boundary state from one GPU to the next)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2303_03848_amd as bsp

    torch.cuda.init()
    log(f"[bench] device {torch.cuda.get_device_name(0)}")
    if args.calibrate_copy > 0:
        # a plain copy of known size, 8 bytes per lane (the solver's access
        # pattern), for scaling the counter readings
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.rand(n + 1, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src[1:], out=dst[1:])
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {n} doubles ({8 * n} bytes read, {8 * n} written)")
        del src, dst
        if args.calibrate_only:
            return

    if args.workload == "large_put":
        out = bench_large_put(args, bsp, torch)
        if not args.no_secondary:
            out["secondary"] = bench_pinn_call(args, bsp, torch, headline=False)
    else:
        out = bench_pinn_call(args, bsp, torch, headline=True)
    if args.all_workloads:
        from bench_workloads import measure_all
        out["other_workloads"] = measure_all(log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
