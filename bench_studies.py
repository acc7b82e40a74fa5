#!/usr/bin/env python
"""Studies around the Parareal solve on one GPU (each prints one JSON line).

  nsweep          speedup against serial fine integration for N = 2 .. 256
                  slices at a fixed total number of fine steps, beside the
                  bound of eq. (8) with the measured c_c, c_f and K
                  (the one-GPU analogue of the paper's Figs. 5-6).
  generalization  Parareal with a network coarse trained for r = 0.03,
                  sigma = 0.4, run at other r and sigma (Sec. 4, Fig. 4):
                  iterations to the tolerance against the training point and
                  against the numerical coarse propagator.
  data_coarse     the same network trained on fine-propagator data alone
                  (no PDE terms) against the physics-informed one and the
                  numerical coarse propagator (Sec. 4, Fig. 3).
  flowmap         a flow-map network coarse (Sec. 3.3's interface: slice
                  start and end, the state, the asset price) fitted to
                  fine-propagator data, against the numerical coarse.

Every number comes from the library's kernels; training runs through the
hand-written loss-and-gradient kernel.  The fine reference is serial fine
integration on the same GPU (one system, all steps in one launch).

Usage: python bench_studies.py nsweep|generalization|data_coarse|flowmap [options]
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def eq8_bound(K: int, N: int, c_c: float, c_f: float) -> float:
    """Speedup bound of eq. (8) with P = N processes, K iterations, coarse
    cost c_c and fine cost c_f per slice."""
    return 1.0 / ((1.0 + K / N) * c_c / c_f + K / N)


def nsweep_splits(total_steps: int, n_values):
    """(N, fine steps per slice) with N * steps = total_steps for each N that
    divides it."""
    return [(N, total_steps // N) for N in n_values if N >= 2 and total_steps % N == 0]


def iterations_to(defects, tol: float):
    """First iteration (1-based) whose defect is <= tol, or None."""
    for k, d in enumerate(defects, 1):
        if d <= tol:
            return k
    return None


# ------------------------------------------------------------------ helpers

def _serial_fine(bsp, torch, p, M, tau_end, steps, u0=None):
    """Serial fine integration on one system from tau = 0: (U at tau_end, ms)."""
    u = bsp.bs_initial(p, M).reshape(1, M) if u0 is None else u0.reshape(1, M).clone()
    tau0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = bsp.bs_fine_propagate_batch(p, M, tau0, tau_end, steps, u)
    torch.cuda.synchronize()
    return out.reshape(M), 1e3 * (time.perf_counter() - t0)


def _fine_levels(bsp, torch, p, M, N, Sf):
    """Serial fine solution at every slice boundary: [N+1, M] (level-by-level
    launches of the fine propagator, Sf steps each)."""
    U = torch.empty((N + 1, M), dtype=torch.float64, device="cuda")
    U[0] = bsp.bs_initial(p, M)
    dT = p["T"] / N
    for n in range(N):
        tau = torch.full((1,), n * dT, dtype=torch.float64, device="cuda")
        U[n + 1] = bsp.bs_fine_propagate_batch(p, M, tau, dT, Sf, U[n].reshape(1, M)).reshape(M)
    return U


def _nl2(a, b):
    """Normalised l2 distance ||a - b|| / ||b|| over all entries."""
    return float((a - b).norm() / b.norm())


def _solve_timed(bsp, torch, pr, tol, reps):
    it, d, _ = pr.solve(tol)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        it, d, _ = pr.solve(tol)
    torch.cuda.synchronize()
    return it, d, 1e3 * (time.perf_counter() - t0) / reps


# ------------------------------------------------------------------ nsweep

def study_nsweep(args, bsp, torch):
    from workloads import LARGE_PUT, option_params
    cfg = LARGE_PUT
    p = option_params(cfg)
    M, tol = cfg["M"], cfg["tol"]
    total = cfg["N"] * cfg["fine_steps"] if args.total_steps <= 0 else args.total_steps
    net = None
    if args.network:
        from paper_2303_03848_amd.pinn import train
        t0 = time.time()
        net, info = train(p, cfg["n_in"], cfg["depth"], cfg["width"], bsp.PREC_FP32,
                          epochs_hi=190, epochs_lo=60)
        net.precision = bsp.PREC_BF16
        log(f"[nsweep] 6x256 network trained in {time.time() - t0:.1f}s")
    _, serial_ms = _serial_fine(bsp, torch, p, M, p["T"], total)
    U_ref, serial_ms2 = _serial_fine(bsp, torch, p, M, p["T"], total)
    serial_ms = min(serial_ms, serial_ms2)
    log(f"[nsweep] serial fine: {total} steps on {M} nodes in {serial_ms:.1f} ms")
    rows = []
    kinds = [("ie", bsp.COARSE_IE, None)] + ([("pinn_ie", bsp.COARSE_PINN_IE, net)] if net else [])
    for N, Sf in nsweep_splits(total, args.n_values):
        for name, kind, nn in kinds:
            pr = bsp.Parareal(p, M, N, Sf, 1, kind, nn)
            it, d, ms = _solve_timed(bsp, torch, pr, tol, 1 if N < 16 else 2)
            err = float((pr.U[N] - U_ref).abs().max())
            # c_f: one fine launch over all N slices; c_c: the sweep's time per
            # slice (one iteration, launch after launch)
            pr.start()
            bsp.bs_profile_enable(True)
            pr.iterate(1)
            pf = bsp.bs_profile_read()
            bsp.bs_profile_enable(False)
            c_f = pf["fine_ms"] / max(pf["fine_launches"], 1)
            c_c = pf["sweep_ms"] / max(pf["sweep_launches"], 1) / N
            s = serial_ms / ms
            row = {"N": N, "fine_steps": Sf, "coarse": name, "iters": it,
                   "time_to_solution_ms": ms, "speedup": s, "efficiency": s / N,
                   "c_f_ms": c_f, "c_c_ms": c_c, "bound_eq8": eq8_bound(it, N, c_c, c_f),
                   "max_error_vs_serial_fine": err, "last_defect": d[-1]}
            rows.append(row)
            log(f"[nsweep] N={N:3d} Sf={Sf:6d} {name:7s}: K={it:3d} {ms:9.2f} ms speedup "
                f"{s:6.2f} (eq. 8: {row['bound_eq8']:6.2f}) err {err:.2e}")
            del pr
    return {"study": "nsweep", "workload": cfg["name"], "M": M, "total_fine_steps": total,
            "tol": tol, "serial_fine_ms": serial_ms, "rows": rows}


# ------------------------------------------------------------ generalization

def study_generalization(args, bsp, torch):
    from workloads import PINN_CALL, SMALL_CALL, option_params
    from paper_2303_03848_amd.pinn import train
    base = option_params(SMALL_CALL)
    base.update(r=0.03, sigma=0.4)  # the training parameters
    t0 = time.time()
    net, info = train(base, PINN_CALL["n_in"], PINN_CALL["depth"], PINN_CALL["width"],
                      bsp.PREC_FP32, epochs_hi=args.epochs[0], epochs_lo=args.epochs[1])
    info = {k: v for k, v in info.items() if k != "history"}
    log(f"[generalization] 4x64 network trained at r=0.03, sigma=0.4 in {time.time() - t0:.1f}s")
    grids = {"small_call_grid": (SMALL_CALL["M"], SMALL_CALL["N"], SMALL_CALL["fine_steps"]),
             "pinn_call_grid": (PINN_CALL["M"], PINN_CALL["N"], PINN_CALL["fine_steps"])}
    tols = (1e-8, 1e-10)
    cases = [("r", f) for f in args.factors] + [("sigma", f) for f in args.factors if f != 1.0]
    out_grids = {}
    for gname, (M, N, Sf) in grids.items():
        rows = []
        for which, f in cases:
            p = dict(base)
            p[which] = base[which] * f
            U_ref = _fine_levels(bsp, torch, p, M, N, Sf)
            row = {"param": which, "factor": f, "r": p["r"], "sigma": p["sigma"]}
            for cname, kind, prec in (("ie", bsp.COARSE_IE, None),
                                      ("pinn_ie_bf16", bsp.COARSE_PINN_IE, bsp.PREC_BF16),
                                      ("pinn_ie_fp32", bsp.COARSE_PINN_IE, bsp.PREC_FP32)):
                nn = None if prec is None else bsp.PinnNet(net.params, net.n_in, net.depth,
                                                           net.width, prec)
                pr = bsp.Parareal(p, M, N, Sf, 1, kind, nn)
                it, d, _ = pr.solve(0.0, max_iter=N)
                err_k = []
                pr.start()
                err_k.append(_nl2(pr.U, U_ref))
                for k in range(1, N + 1):
                    pr.iterate(k)
                    err_k.append(_nl2(pr.U, U_ref))
                row[cname] = {"iters_to": {str(t): iterations_to(d, t) for t in tols},
                              "defects": d, "nl2_error_vs_fine_by_iteration": err_k}
            rows.append(row)
            log(f"[generalization] {gname} {which} x{f}: iterations to 1e-10: IE "
                f"{row['ie']['iters_to']['1e-10']}, PINN_IE bf16 "
                f"{row['pinn_ie_bf16']['iters_to']['1e-10']}, fp32 "
                f"{row['pinn_ie_fp32']['iters_to']['1e-10']}")
        out_grids[gname] = {"M": M, "N": N, "fine_steps": Sf, "rows": rows}
    return {"study": "generalization", "trained_at": {"r": 0.03, "sigma": 0.4},
            "option": {k: base[k] for k in ("K", "T", "s_max", "is_put")},
            "network": "4x64 tanh", "training": info, "grids": out_grids}


# --------------------------------------------------------------- data_coarse

def study_data_coarse(args, bsp, torch):
    from workloads import PINN_CALL, option_params
    from paper_2303_03848_amd.pinn import train, train_on_data
    cfg = PINN_CALL
    p = option_params(cfg)
    M, Sf_total = cfg["M"], cfg["N"] * cfg["fine_steps"]
    # training data: the serial fine trajectory at `levels` equally spaced
    # times (fine steps between them), every node, v = V/K at (tau, S/K)
    levels = args.data_levels
    U_data = _fine_levels(bsp, torch, p, M, levels, Sf_total // levels)
    S = torch.arange(1, M + 1, dtype=torch.float64, device="cuda") * (p["s_max"] / (M + 1))
    taus = torch.arange(levels + 1, dtype=torch.float64, device="cuda") * (p["T"] / levels)
    X = torch.stack([taus[:, None].expand(-1, M).reshape(-1),
                     (S / p["K"])[None, :].expand(levels + 1, -1).reshape(-1)], 1).float()
    y = (U_data / p["K"]).reshape(-1).float()
    t0 = time.time()
    nn_data, info_d = train_on_data(p, X, y, cfg["n_in"], cfg["depth"], cfg["width"],
                                    epochs_hi=args.epochs[0], epochs_lo=args.epochs[1])
    log(f"[data_coarse] data-only network trained in {time.time() - t0:.1f}s: {info_d}")
    t0 = time.time()
    nn_pinn, info_p = train(p, cfg["n_in"], cfg["depth"], cfg["width"], bsp.PREC_FP32,
                            epochs_hi=args.epochs[0], epochs_lo=args.epochs[1])
    info_p = {k: v for k, v in info_p.items() if k != "history"}
    log(f"[data_coarse] physics-informed network trained in {time.time() - t0:.1f}s")
    out_n = {}
    for N in args.slices:
        Sf = Sf_total // N
        U_ref = _fine_levels(bsp, torch, p, M, N, Sf)
        res = {}
        for cname, kind, net in (("ie", bsp.COARSE_IE, None),
                                 ("nn_data_pinn_ie", bsp.COARSE_PINN_IE, nn_data),
                                 ("pinn_pinn_ie", bsp.COARSE_PINN_IE, nn_pinn),
                                 ("nn_data_direct", bsp.COARSE_PINN, nn_data),
                                 ("pinn_direct", bsp.COARSE_PINN, nn_pinn)):
            for prec in ((None,) if net is None else (bsp.PREC_BF16, bsp.PREC_FP32)):
                nn = None if net is None else bsp.PinnNet(net.params, net.n_in, net.depth,
                                                          net.width, prec)
                key = cname if prec is None else cname + ("_bf16" if prec == bsp.PREC_BF16
                                                          else "_fp32")
                pr = bsp.Parareal(p, M, N, Sf, 1, kind, nn)
                it, d, ms = _solve_timed(bsp, torch, pr, cfg["tol"], 3)
                pr.start()
                # coarse prediction (iteration 0) against the fine solution,
                # level by level, then the iteration errors
                coarse_err = [float((pr.U[n] - U_ref[n]).norm() / U_ref[n].norm())
                              for n in range(1, N + 1)]
                err_k = [_nl2(pr.U, U_ref)]
                for k in range(1, min(it, N) + 1):
                    pr.iterate(k)
                    err_k.append(_nl2(pr.U, U_ref))
                res[key] = {"iters": it, "time_to_solution_ms": ms, "first_defect": d[0],
                            "coarse_nl2_error_by_level": coarse_err,
                            "nl2_error_vs_fine_by_iteration": err_k}
                log(f"[data_coarse] N={N} {key}: K={it} {ms:.3f} ms, coarse error at T "
                    f"{coarse_err[-1]:.2e}, first defect {d[0]:.3e}")
        out_n[str(N)] = {"fine_steps": Sf, "coarse": res}
    return {"study": "data_coarse", "workload": cfg["name"], "M": M, "tol": cfg["tol"],
            "data": {"levels": levels, "points": int(X.shape[0]),
                     "source": "serial fine propagator on the same grid"},
            "training_data_only": info_d, "training_physics": info_p, "slices": out_n}


# ------------------------------------------------------------------ flowmap

def study_flowmap(args, bsp, torch):
    """A flow-map network coarse: w(tau_s, tau_e, V_s/K, S/K) -> V_e/K fitted
    to fine-propagator data (the paper gives no loss for this interface):
    states from the serial fine trajectory and from the first iterates of
    Parareal with the numerical coarse, each propagated over its slice by the
    fine propagator; then Parareal with it against the numerical coarse."""
    from workloads import PINN_CALL, option_params
    from paper_2303_03848_amd.pinn import train_on_data
    cfg = PINN_CALL
    p = option_params(cfg)
    M, N, Sf, tol = cfg["M"], cfg["N"], cfg["fine_steps"], cfg["tol"]
    dT = p["T"] / N
    states = [_fine_levels(bsp, torch, p, M, N, Sf)[:N]]
    pr = bsp.Parareal(p, M, N, Sf, 1, bsp.COARSE_IE)
    states.append(pr.start()[:N].clone())
    for k in range(1, args.iterate_states + 1):
        pr.iterate(k)
        states.append(pr.U[:N].clone())
    S = torch.arange(1, M + 1, dtype=torch.float64, device="cuda") * (p["s_max"] / (M + 1))
    tau0 = torch.arange(N, dtype=torch.float64, device="cuda") * dT
    Xs, ys = [], []
    for U in states:
        Fv = bsp.bs_fine_propagate_batch(p, M, tau0, dT, Sf, U.contiguous())
        X = torch.stack([tau0[:, None].expand(-1, M), (tau0 + dT)[:, None].expand(-1, M),
                         U / p["K"], (S / p["K"])[None, :].expand(N, -1)], 2).reshape(-1, 4)
        Xs.append(X.float())
        ys.append((Fv / p["K"]).reshape(-1).float())
    X, y = torch.cat(Xs), torch.cat(ys)
    t0 = time.time()
    net, info = train_on_data(p, X, y, 4, cfg["depth"], cfg["width"],
                              epochs_hi=args.epochs[0], epochs_lo=args.epochs[1])
    log(f"[flowmap] 4-input network fitted to {X.shape[0]} fine-propagator pairs in "
        f"{time.time() - t0:.1f}s: {info}")
    U_ref = _fine_levels(bsp, torch, p, M, N, Sf)
    res = {}
    for name, kind, prec in (("ie", bsp.COARSE_IE, None),
                             ("flowmap_fp32", bsp.COARSE_FLOWMAP, bsp.PREC_FP32),
                             ("flowmap_bf16", bsp.COARSE_FLOWMAP, bsp.PREC_BF16)):
        nn = None if prec is None else bsp.PinnNet(net.params, 4, net.depth, net.width, prec)
        q = bsp.Parareal(p, M, N, Sf, 1, kind, nn)
        it, d, ms = _solve_timed(bsp, torch, q, tol, 3)
        q.start()
        coarse_err = [float((q.U[n] - U_ref[n]).norm() / U_ref[n].norm()) for n in range(1, N + 1)]
        res[name] = {"iters": it, "time_to_solution_ms": ms, "first_defect": d[0],
                     "defects": d, "coarse_nl2_error_by_level": coarse_err}
        log(f"[flowmap] {name}: K={it} {ms:.3f} ms, first defect {d[0]:.3e}, coarse error at T "
            f"{coarse_err[-1]:.2e}")
    return {"study": "flowmap", "workload": cfg["name"], "M": M, "N": N, "fine_steps": Sf,
            "tol": tol, "training": dict(info, pairs=int(X.shape[0]),
                                         state_sets=len(states)),
            "network": f"{cfg['depth']}x{cfg['width']} tanh, inputs (tau_s, tau_e, V_s/K, S/K)",
            "coarse": res}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="study", required=True)
    a = sub.add_parser("nsweep")
    a.add_argument("--n-values", type=int, nargs="+", default=[2, 4, 8, 16, 32, 64, 128, 256])
    a.add_argument("--total-steps", type=int, default=0,
                   help="fine steps over [0, T] (default: the 16384-node put's 256 x 2048)")
    a.add_argument("--network", action="store_true",
                   help="also run the network coarse (6 x 256, trained first)")
    g = sub.add_parser("generalization")
    g.add_argument("--factors", type=float, nargs="+", default=[0.5, 1.0, 2.0, 5.0, 10.0, 12.0])
    g.add_argument("--epochs", type=int, nargs=2, default=(5000, 800))
    d = sub.add_parser("data_coarse")
    d.add_argument("--epochs", type=int, nargs=2, default=(5000, 800))
    d.add_argument("--data-levels", type=int, default=128)
    d.add_argument("--slices", type=int, nargs="+", default=[16, 32])
    f = sub.add_parser("flowmap")
    f.add_argument("--epochs", type=int, nargs=2, default=(1500, 300))
    f.add_argument("--iterate-states", type=int, default=2,
                   help="iterates of the numerical-coarse Parareal added to the training states")
    args = ap.parse_args()

    import torch
    import paper_2303_03848_amd as bsp
    torch.cuda.init()
    fn = {"nsweep": study_nsweep, "generalization": study_generalization,
          "data_coarse": study_data_coarse, "flowmap": study_flowmap}[args.study]
    print(json.dumps(fn(args, bsp, torch)), flush=True)


if __name__ == "__main__":
    main()
