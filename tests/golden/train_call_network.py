"""Train the 4 x 64 tanh call network of the 1024-node workload with the
FP64 oracle alone (oracle/mlp.py loss and hand-written gradient, plain Adam
in numpy), and store its weights as a test fixture.

The GPU tests use these weights as a trained network whose values never came
from the HIP path: the network coarse propagator is evaluated by the GPU in
FP32 / BF16 and by the oracle in FP64 from the same weights.

Recipe (Sec. 3.3 of the paper, with the readings of the tests' workloads):
fixed uniform collocation sets (65536 interior, 4096 terminal, 2048 boundary
points), reshuffled every epoch into minibatches of 8192 / 512 / 256 (8 steps
per epoch); Adam (beta1 0.9, beta2 0.999, eps 1e-8) at learning rate 1e-2 for
5000 epochs, then 1e-3 for 800 epochs; Xavier-normal initialisation with
seed 0.

Usage: python -m tests.golden.train_call_network [--epochs HI LO] [--out PATH]
Writes PATH (float32 .npy, torch nn.Linear packing) and PATH with .json
(recipe and final loss terms).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import mlp  # noqa: E402
from workloads import (PINN_CALL, SEED, collocation, minibatch_indices, option_params,  # noqa: E402
                       xavier_normal)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pinn_call_4x64.npy")


def adam_train(cfg, epochs_hi, epochs_lo, seed=SEED, init_seed=0, batch=(8192, 512, 256),
               sizes=(65536, 4096, 2048), log=print):
    p = option_params(cfg)
    n_in, depth, width = cfg["n_in"], cfg["depth"], cfg["width"]
    Xf, Xe, Xb = collocation(*sizes, p["T"], p["s_max"] / p["K"], seed=seed)
    theta = xavier_normal(n_in, depth, width, init_seed).astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    b1, b2, eps = 0.9, 0.999, 1e-8
    step = 0
    t0 = time.time()
    per_epoch = min(sizes[0] // batch[0], sizes[1] // batch[1], sizes[2] // batch[2])
    for epoch in range(epochs_hi + epochs_lo):
        lr = 1e-2 if epoch < epochs_hi else 1e-3
        idx_f = minibatch_indices(sizes[0], batch[0], epoch, seed)
        idx_e = minibatch_indices(sizes[1], batch[1], epoch, seed + 1)
        idx_b = minibatch_indices(sizes[2], batch[2], epoch, seed + 2)
        for q in range(per_epoch):
            g = mlp.loss_grad(theta, Xf[idx_f[q]], Xe[idx_e[q]], Xb[idx_b[q]], n_in, depth, width,
                              p["is_put"], p["sigma"], p["r"])
            step += 1
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            mh = m / (1 - b1 ** step)
            vh = v / (1 - b2 ** step)
            theta = theta - lr * mh / (np.sqrt(vh) + eps)
        if (epoch + 1) % 100 == 0:
            l3 = mlp.loss3(theta, Xf[:8192], Xe[:512], Xb[:256], n_in, depth, width, p["is_put"],
                           p["sigma"], p["r"])
            log(f"epoch {epoch + 1}: loss {sum(l3):.3e} {l3} ({time.time() - t0:.0f} s)")
    l3 = mlp.loss3(theta, Xf, Xe, Xb, n_in, depth, width, p["is_put"], p["sigma"], p["r"])
    return theta, {"epochs": [epochs_hi, epochs_lo], "steps": step, "lr": [1e-2, 1e-3],
                   "batch": list(batch), "sizes": list(sizes), "seed": seed,
                   "init_seed": init_seed, "final_loss3_all_points": [float(x) for x in l3],
                   "seconds": time.time() - t0, "workload": cfg["name"],
                   "network": f"{depth}x{width} tanh, inputs (tau, S/K)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, nargs=2, default=(5000, 800))
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    theta, info = adam_train(PINN_CALL, *a.epochs, log=lambda s: print(s, flush=True))
    np.save(a.out, theta.astype(np.float32))
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump(info, f, indent=1)
    print("wrote", a.out, info["final_loss3_all_points"], flush=True)


if __name__ == "__main__":
    main()
