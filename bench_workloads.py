"""Measurements of the workloads besides the headline ones (one GPU): the
small call, one training step of the residual loss and the batch of 512
options.  Used by ``bench.py --all-workloads``; every number comes from the
library's kernels, timed after a warm-up.
"""
from __future__ import annotations

import time

import numpy as np
import torch

import paper_2303_03848_amd as bsp
from workloads import (OPTION_BATCH, SMALL_CALL, TRAIN_STEP, collocation, option_batch,
                       option_params, xavier_normal)

FP32_VALU_PEAK = 157.3e12
BF16_MFMA_PEAK = 2.5e15


def _timed(fn, reps: int) -> float:
    """Mean milliseconds of fn() over reps calls after one warm-up call."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def parareal_cells(M: int, N: int, Sf: int, iters: int) -> float:
    """Fine cell-updates of a Parareal solve of `iters` iterations (slices
    n < k-1 are not propagated in iteration k)."""
    return float(sum((N - min(k - 1, N - 1)) * Sf * M for k in range(1, iters + 1)))


def small_call() -> dict:
    cfg = SMALL_CALL
    p, M, N, Sf = option_params(cfg), cfg["M"], cfg["N"], cfg["fine_steps"]
    pr = bsp.Parareal(p, M, N, Sf, 1, bsp.COARSE_IE)
    it = [0]

    def solve():
        it[0] = pr.solve(cfg["tol"])[0]

    ms = _timed(solve, 20)
    return {"workload": cfg["name"], "coarse": "implicit_euler", "time_to_solution_ms": ms,
            "iters": it[0], "cell_updates_per_s": parareal_cells(M, N, Sf, it[0]) / (ms / 1e3)}


def train_step() -> dict:
    """One minibatch of the residual loss, forward and hand-written backward
    (no optimiser update), FP32 and BF16-MFMA."""
    cfg = TRAIN_STEP
    p = option_params(cfg)
    d, w = cfg["depth"], cfg["width"]
    nf, ne, nb = cfg["batch_f"], cfg["batch_e"], cfg["batch_b"]
    Xf, Xe, Xb = collocation(nf, ne, nb, p["T"], p["s_max"] / p["K"])
    Xf, Xe, Xb = (torch.tensor(a, dtype=torch.float32, device="cuda") for a in (Xf, Xe, Xb))
    theta = torch.tensor(xavier_normal(cfg["n_in"], d, w, 0), device="cuda")
    # algorithmic flops: 4 derivative streams forward and 2x backward for the
    # interior points, the value stream for terminal and boundary points,
    # through the (d - 1) hidden w x w products
    flops = 3 * 2 * w * w * (d - 1) * (4 * nf + ne + nb)
    out = {"workload": cfg["name"], "network": f"{d}x{w} tanh",
           "points": [nf, ne, nb], "flops_per_step": flops}
    for name, prec, peak in (("fp32", bsp.PREC_FP32, FP32_VALU_PEAK),
                             ("bf16", bsp.PREC_BF16, BF16_MFMA_PEAK)):
        net = bsp.PinnNet(theta, cfg["n_in"], d, w, prec)
        ws = torch.empty(bsp.pinn_residual_workspace_size(net, nf, ne, nb), dtype=torch.uint8,
                         device="cuda")
        loss3 = torch.empty(3, dtype=torch.float32, device="cuda")
        grad = torch.empty_like(theta)
        ms = _timed(lambda: bsp.pinn_residual_fwd_bwd(net, p, Xf, Xe, Xb, ws, loss3, grad), 50)
        out[name] = {"ms_per_step": ms, "tflops": flops / (ms / 1e3) / 1e12,
                     "frac_of_peak": flops / (ms / 1e3) / peak,
                     "peak": "FP32 vector 157.3 TFLOP/s" if name == "fp32"
                     else "BF16 dense MFMA 2.5 PFLOP/s"}
    return out


def train_batch_network(epochs=(1000, 200), precision: int = bsp.PREC_BF16):
    """The parametric network of the batch: (tau, S/K, sigma, r) -> V/K of a
    call, trained over the batch's box of maturities, S/K, sigma and r (puts
    take put-call parity on the device).  FP32 training, evaluated in
    `precision`."""
    from paper_2303_03848_amd.pinn import train
    cfg = OPTION_BATCH
    box = dict(K=1.0, r=0.0, sigma=0.2, T=cfg["T_range"][1], s_max=cfg["s_max_over_K"],
               is_put=False)
    net, info = train(box, cfg["n_in"], cfg["depth"], cfg["width"], bsp.PREC_FP32,
                      epochs_hi=epochs[0], epochs_lo=epochs[1],
                      coeff_box=(cfg["sigma_range"], cfg["r_range"]))
    net.precision = precision
    return net, {k: v for k, v in info.items() if k != "history"}


def batch_options(n_opt: int | None = None, train_epochs=(1000, 200)) -> dict:
    """The batch of options: numerical coarse, and the network coarse with
    the parametric network in BF16 (one launch per phase and block shape,
    iterations queued ahead of the host's convergence check)."""
    cfg = OPTION_BATCH
    opts = option_batch(cfg, n_opt=n_opt)
    for o in opts:
        o["fine_steps"] = cfg["fine_steps"]
        o["coarse_steps"] = cfg["coarse_steps"]
    serial = sum(float(o["N"] * o["fine_steps"] * o["M"]) for o in opts)

    def run(kind, net):
        res = {}

        def solve():
            _, _, iters, _, _ = bsp.parareal_solve_batch(opts, kind, cfg["tol"], net=net)
            res["iters"] = iters

        ms = _timed(solve, 2)
        iters = np.array(res["iters"])
        cells = sum(parareal_cells(o["M"], o["N"], o["fine_steps"], int(k))
                    for o, k in zip(opts, iters))
        return {"time_ms": ms, "iters_mean": float(iters.mean()), "iters_min": int(iters.min()),
                "iters_max": int(iters.max()), "cell_updates_per_s": cells / (ms / 1e3)}

    out = {"workload": cfg["name"], "options": len(opts), "serial_fine_cells": serial,
           "numeric_coarse_default_shapes": run(bsp.COARSE_IE, None)}
    # block shapes per grid size picked by the autotuner on this batch
    from paper_2303_03848_amd.autotune import tune_batch
    t0 = time.time()
    shapes = tune_batch(cfg["name"], opts, use_cache=False)
    out["tuned_shapes"] = {M: {"fine": e["fine"], "sweep": e["sweep"]} for M, e in shapes.items()}
    out["tuning_s"] = time.time() - t0
    out["numeric_coarse"] = run(bsp.COARSE_IE, None)
    if train_epochs:
        t0 = time.time()
        net, info = train_batch_network(train_epochs)
        out["network_training"] = dict(info, wall_s=time.time() - t0)
        out["network_coarse_bf16"] = run(bsp.COARSE_PINN_IE, net)
        out["network"] = f"{cfg['depth']}x{cfg['width']} tanh, inputs (tau, S/K, sigma, r), bf16"
    bsp.bs_tune_reset()
    return out


def measure_all(log=print) -> dict:
    out = {}
    for name, fn in (("small_call", small_call), ("train_step", train_step),
                     ("option_batch", batch_options)):
        t0 = time.time()
        out[name] = fn()
        log(f"[workloads] {name}: {time.time() - t0:.1f}s {out[name]}")
    return out


def main():
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="measure the non-headline workloads (one GPU)")
    ap.add_argument("--only", choices=["small_call", "train_step", "option_batch"], action="append",
                    help="run only these (repeatable); default: all")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain elementwise copy of MIB MiB (float64) so a counter "
                         "profile of this command has a copy kernel of known size")
    args = ap.parse_args()
    torch.cuda.init()
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.rand(n + 1, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src[1:], out=dst[1:])
        torch.cuda.synchronize()
        del src, dst
    fns = {"small_call": small_call, "train_step": train_step, "option_batch": batch_options}
    out = {}
    for name in args.only or list(fns):
        t0 = time.time()
        out[name] = fns[name]()
        print(f"[workloads] {name}: {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
