"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the
benchmark.

This module only draws numbers and names workloads: it holds none of the
method's arithmetic (no payoff, boundary data, operator or network maths),
so both the oracle and the HIP path can take their inputs from it without
sharing any of the computation.

Workloads (the option parameters, grids and slice counts each run uses):
  * ``SMALL_CALL``  European call K=100, r=0.05, sigma=0.2, T=1, S in [0, 300],
    M=256 interior nodes, N=8 slices, 64 Crank-Nicolson steps per slice,
    1 implicit-Euler step per slice, tol 1e-8.
  * ``PINN_CALL``   the same call with M=1024, N=32, 512 CN steps per slice,
    a 4 x 64 tanh network (tau, S/K) -> V/K.
  * ``TRAIN_STEP``  65536 interior, 4096 terminal, 2048 boundary points,
    128 x 4 tanh network, minibatches of 8192 / 512 / 256 points.
  * ``OPTION_BATCH`` 512 calls and puts with drawn coefficients, grids and
    slice counts, 256 CN steps per slice, parametrised 128 x 4 network.
  * ``LARGE_PUT``   put K=100, r=0.03, sigma=0.35, T=2, S in [0, 400],
    M=16384, N=256, 2048 CN steps per slice, 256 x 6 network, tol 1e-10.
"""
from __future__ import annotations

import numpy as np

SEED = 2303_03848

SMALL_CALL = dict(name="small_call_M256_N8", K=100.0, r=0.05, sigma=0.2, T=1.0, s_max=300.0,
                  is_put=False, M=256, N=8, fine_steps=64, coarse_steps=1, tol=1e-8,
                  payoff_mode=1)

PINN_CALL = dict(name="pinn_call_M1024_N32", K=100.0, r=0.05, sigma=0.2, T=1.0, s_max=300.0,
                 is_put=False, M=1024, N=32, fine_steps=512, coarse_steps=1, tol=1e-8,
                 payoff_mode=1, n_in=2, depth=4, width=64)

TRAIN_STEP = dict(name="pinn_train_w128x4", K=100.0, r=0.05, sigma=0.2, T=1.0, s_max=300.0,
                  is_put=False, n_in=2, depth=4, width=128, n_f=65536, n_e=4096, n_b=2048,
                  batch_f=8192, batch_e=512, batch_b=256)

OPTION_BATCH = dict(name="option_batch_512", n_opt=512, fine_steps=256, coarse_steps=1, tol=1e-8,
                    payoff_mode=1, M_choices=(256, 512, 1024, 2048, 4096), N_range=(16, 64),
                    sigma_range=(0.1, 0.5), r_range=(0.0, 0.1), K_range=(50.0, 150.0),
                    T_range=(0.25, 2.0), s_max_over_K=4.0, n_in=4, depth=4, width=128)

LARGE_PUT = dict(name="large_put_M16384_N256", K=100.0, r=0.03, sigma=0.35, T=2.0, s_max=400.0,
                 is_put=True, M=16384, N=256, fine_steps=2048, coarse_steps=1, tol=1e-10,
                 payoff_mode=1, n_in=2, depth=6, width=256)


def option_params(cfg: dict) -> dict:
    """The option fields of a workload dict."""
    return {k: cfg[k] for k in ("K", "r", "sigma", "T", "s_max", "is_put")}


def xavier_normal(n_in: int, depth: int, width: int, seed: int = 0) -> np.ndarray:
    """Flat float32 parameters in torch nn.Linear order, weights drawn
    N(0, 2/(fan_in + fan_out)), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    fan_in = n_in
    for _ in range(depth):
        std = np.sqrt(2.0 / (fan_in + width))
        parts.append(rng.normal(0.0, std, size=width * fan_in))
        parts.append(np.zeros(width))
        fan_in = width
    std = np.sqrt(2.0 / (width + 1))
    parts.append(rng.normal(0.0, std, size=width))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)


def perturbed(params: np.ndarray, scale: float, seed: int = 1) -> np.ndarray:
    """params + scale * N(0,1) noise (float32): gives non-zero biases for tests."""
    rng = np.random.default_rng(seed)
    return (params.astype(np.float64) + scale * rng.normal(size=params.size)).astype(np.float32)


def collocation(n_f: int, n_e: int, n_b: int, tau_max: float, x_max: float, seed: int = SEED,
                coeff_box=None):
    """Collocation points in (tau, x = S/K), uniform draws:
      interior (tau, x) ~ U[0, tau_max] x U[0, x_max];
      terminal tau = 0, x ~ U[0, x_max];
      boundary tau ~ U[0, tau_max], half at x = 0 and half at x = x_max.
    With coeff_box = ((sig_lo, sig_hi), (r_lo, r_hi)) two more columns
    sigma ~ U, r ~ U are appended (network parametrised by the coefficients).
    Returns float64 arrays X_f [n_f, c], X_e [n_e, c], X_b [n_b, c]."""
    rng = np.random.default_rng(seed)
    X_f = np.stack([rng.uniform(0.0, tau_max, n_f), rng.uniform(0.0, x_max, n_f)], axis=1)
    X_e = np.stack([np.zeros(n_e), rng.uniform(0.0, x_max, n_e)], axis=1)
    half = n_b // 2
    xb = np.concatenate([np.zeros(half), np.full(n_b - half, x_max)])
    X_b = np.stack([rng.uniform(0.0, tau_max, n_b), xb], axis=1)
    if coeff_box is not None:
        (s0, s1), (r0, r1) = coeff_box
        def extra(n):
            return np.stack([rng.uniform(s0, s1, n), rng.uniform(r0, r1, n)], axis=1)
        X_f = np.concatenate([X_f, extra(n_f)], axis=1)
        X_e = np.concatenate([X_e, extra(n_e)], axis=1)
        X_b = np.concatenate([X_b, extra(n_b)], axis=1)
    return X_f, X_e, X_b


def minibatch_indices(n: int, batch: int, epoch: int, seed: int = SEED):
    """Per-epoch permutation of range(n), split into consecutive batches."""
    perm = np.random.default_rng(seed + 7919 * (epoch + 1)).permutation(n)
    return [perm[i:i + batch] for i in range(0, n - batch + 1, batch)]


def option_batch(cfg: dict = OPTION_BATCH, seed: int = SEED, n_opt: int | None = None):
    """Draw the option table of the batched workload: a list of dicts with
    K, r, sigma, T, s_max, is_put, M, N."""
    rng = np.random.default_rng(seed)
    n = cfg["n_opt"] if n_opt is None else n_opt
    out = []
    for i in range(n):
        K = rng.uniform(*cfg["K_range"])
        out.append(dict(
            K=float(K), r=float(rng.uniform(*cfg["r_range"])),
            sigma=float(rng.uniform(*cfg["sigma_range"])), T=float(rng.uniform(*cfg["T_range"])),
            s_max=float(cfg["s_max_over_K"] * K), is_put=bool(i % 2),
            M=int(rng.choice(cfg["M_choices"])),
            N=int(rng.integers(cfg["N_range"][0], cfg["N_range"][1] + 1))))
    return out


def random_states(nsys: int, M: int, scale: float = 100.0, seed: int = 3) -> np.ndarray:
    """Smooth-plus-noise float64 states [nsys, M] for propagator checks."""
    rng = np.random.default_rng(seed)
    j = np.linspace(0.0, 1.0, M)
    base = scale * np.maximum(3.0 * j - 1.0, 0.0)
    return base[None, :] + scale * 0.01 * rng.normal(size=(nsys, M))
