"""Serial fine solution of the 16384-node put (the fixed point of eq. (7),
Sec. 3.1: U_{n+1} = F(U_n), n = 0..N-1, with F = 2048 Crank-Nicolson steps
per slice, Sec. 3.2), computed by the FP64 oracle alone and stored at a few
time levels as a test fixture.

The integration is serial over the 256 slices (each level needs the one
before), about 20 minutes of one CPU core: too long for the body of a GPU
test, so the levels the tests compare are stored.  Every level is a plain
oracle result; nothing here comes from the HIP library.

Usage: python -m tests.golden.large_put_reference [--out PATH]
Writes PATH (.npz: `levels` [L] int, `U` [L][M] float64, and the workload's
sizes) and prints the wall time.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import LARGE_PUT, option_params  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_put_levels.npz")
# early levels (rounding of the first slices), powers of two, and the last
# level, which carries everything accumulated across the slices
LEVELS = (0, 1, 2, 4, 8, 16, 32, 64, 128, 192, 255, 256)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    cfg = LARGE_PUT
    p = oracle.params_from(option_params(cfg))
    M, N, Sf = cfg["M"], cfg["N"], cfg["fine_steps"]
    t0 = time.time()
    u = oracle.initial(p, M, cfg["payoff_mode"])
    dT = p.T / N
    keep = {0: u.copy()}
    for n in range(N):
        u = oracle.fine(p, M, n * dT, dT, Sf, u)
        if n + 1 in LEVELS:
            keep[n + 1] = u.copy()
        if (n + 1) % 16 == 0:
            print(f"level {n + 1}/{N} ({time.time() - t0:.0f} s)", flush=True)
    levels = np.array(sorted(keep), dtype=np.int64)
    np.savez_compressed(a.out, levels=levels, U=np.stack([keep[int(n)] for n in levels]),
                        M=M, N=N, fine_steps=Sf)
    print(f"wrote {a.out}: levels {levels.tolist()} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
