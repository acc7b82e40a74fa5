"""Autotuner for the block shapes of the tridiagonal kernels.

Each system is solved by one thread block; the shape (threads per block,
nodes per thread) trades per-step issue time (more nodes per thread) against
exchange rounds between threads (more threads).  The best shape depends on M,
on the number of concurrent systems and on the coupling strength (which sets
how many reduction stages a step needs), so it is measured, not guessed:
every built shape that covers M is timed on the actual workload through the
library's shape override, checked to agree with the default shape, and the
fastest is installed.  Results are cached in a JSON file keyed by device and
workload.
"""
from __future__ import annotations

import json
import os

import torch

import paper_2303_03848_amd as bsp

BUILT_SHAPES = [(64, 2), (64, 4), (64, 8), (64, 16), (128, 4), (128, 8), (128, 16), (256, 4),
                (256, 8), (256, 16), (512, 8)]
FINE, SWEEP = 0, 1
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def candidates(M: int):
    return [(T, MC) for T, MC in BUILT_SHAPES if T * MC >= M and T * MC < 8 * max(M, 64)]


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_fine(p: dict, M: int, nsys: int, steps: int, dtau: float, reps: int = 3):
    """Time the fine propagator on nsys systems for every candidate shape.
    Returns (best (T, MC), {shape: ms})."""
    u = bsp.bs_initial(p, M).repeat(nsys, 1).contiguous()
    tau0 = torch.arange(nsys, dtype=torch.float64, device="cuda") * dtau
    bsp.bs_tune_reset()
    ref = bsp.bs_fine_propagate_batch(p, M, tau0, dtau, steps, u)
    times = {}
    for T, MC in candidates(M):
        bsp.bs_tune_reset()
        bsp.bs_tune_set_shape(FINE, M, M, T, MC)
        out = bsp.bs_fine_propagate_batch(p, M, tau0, dtau, steps, u)
        diff = (out - ref).abs().max().item() / max(ref.abs().max().item(), 1e-300)
        if diff > 1e-11:
            raise RuntimeError(f"shape {(T, MC)} disagrees with the default by {diff:.2e}")
        times[(T, MC)] = _time(lambda: bsp.bs_fine_propagate_batch(p, M, tau0, dtau, steps, u,
                                                                   out), reps)
    bsp.bs_tune_reset()
    best = min(times, key=times.get)
    return best, times


def tune_sweep(p: dict, M: int, N: int, fine_steps: int, kind: int = bsp.COARSE_IE, net=None,
               reps: int = 3, fine_shape=None):
    """Time one Parareal iteration's sweep for every candidate sweep shape
    (the fine kernel takes fine_shape, or its default).  Returns (best,
    {shape: ms})."""
    times = {}
    pr = bsp.Parareal(p, M, N, fine_steps, 1, kind, net)
    for T, MC in candidates(M):
        bsp.bs_tune_reset()
        if fine_shape is not None:
            bsp.bs_tune_set_shape(FINE, M, M, *fine_shape)
        bsp.bs_tune_set_shape(SWEEP, M, M, T, MC)
        pr.start()
        bsp.bs_profile_enable(True)
        for k in range(1, reps + 1):
            pr.iterate(k)
        prof = bsp.bs_profile_read()
        bsp.bs_profile_enable(False)
        times[(T, MC)] = prof["sweep_ms"] / max(prof["sweep_launches"], 1)
    bsp.bs_tune_reset()
    best = min(times, key=times.get)
    return best, times


def _key(name: str) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return f"{dev}|{name}"


def load_cache(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def tune_workload(name: str, p: dict, M: int, N: int, fine_steps: int, use_cache: bool = True,
                  path: str = CACHE, verbose: bool = False):
    """Pick and install the fine and sweep shapes for one Parareal workload."""
    cache = load_cache(path) if use_cache else {}
    key = _key(name)
    if key in cache:
        ent = cache[key]
    else:
        dT = p["T"] / N
        bf, tf = tune_fine(p, M, N, fine_steps, dT)
        bs, ts = tune_sweep(p, M, N, fine_steps, fine_shape=bf)
        ent = {"fine": list(bf), "sweep": list(bs),
               "fine_ms": {f"{a}x{b}": v for (a, b), v in tf.items()},
               "sweep_ms": {f"{a}x{b}": v for (a, b), v in ts.items()}}
        cache[key] = ent
        try:
            with open(path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    bsp.bs_tune_reset()
    bsp.bs_tune_set_shape(FINE, M, M, *ent["fine"])
    bsp.bs_tune_set_shape(SWEEP, M, M, *ent["sweep"])
    if verbose:
        print(f"[autotune] {name}: fine {ent['fine']} sweep {ent['sweep']}", flush=True)
    return ent


def tune_batch(name: str, options, use_cache: bool = True, path: str = CACHE,
               verbose: bool = False):
    """Pick and install the fine and sweep shapes of every grid size of a
    batch of options (the batch solve launches one class per shape): per
    distinct M, the fine shape is timed on as many systems as the batch has
    slices of that M (a representative option's coefficients) and the sweep
    shape on one representative option.  Returns {M: entry}."""
    cache = load_cache(path) if use_cache else {}
    key = _key(name)
    ent = cache.get(key)
    if ent is None:
        ent = {}
        for M in sorted({o["M"] for o in options}):
            group = [o for o in options if o["M"] == M]
            rep = group[len(group) // 2]
            p = {k: rep[k] for k in ("K", "r", "sigma", "T", "s_max", "is_put")}
            nsys = sum(o["N"] for o in group)
            dT = rep["T"] / rep["N"]
            bsp.bs_tune_reset()
            bf, tf = tune_fine(p, M, nsys, rep["fine_steps"], dT)
            bs, ts = tune_sweep(p, M, rep["N"], rep["fine_steps"], fine_shape=bf)
            ent[str(M)] = {"fine": list(bf), "sweep": list(bs), "systems": nsys,
                           "fine_ms": {f"{a}x{b}": v for (a, b), v in tf.items()},
                           "sweep_ms": {f"{a}x{b}": v for (a, b), v in ts.items()}}
        cache[key] = ent
        try:
            with open(path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    bsp.bs_tune_reset()
    for M, e in ent.items():
        bsp.bs_tune_set_shape(FINE, int(M), int(M), *e["fine"])
        bsp.bs_tune_set_shape(SWEEP, int(M), int(M), *e["sweep"])
        if verbose:
            print(f"[autotune] {name} M={M}: fine {e['fine']} sweep {e['sweep']}", flush=True)
    return ent
