"""FP64 oracle for Parareal with a flow-map network as coarse propagator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.3 describes the coarse network's interface: it receives a time slice
[t_start, t_end], the option price at t_start and the asset prices S, and
returns the price at t_end.  Read node by node on the space grid (in time to
maturity tau):

    G(U_n)[j] = K * w(tau_n, tau_{n+1}, U_n[j] / K, S_j / K),

with w a network of 4 inputs (mlp.forward, FP64).  Parareal is eq. (7) in
plain loops: k = 0 the coarse prediction slice after slice; iteration k
propagates every slice with the fine propagator (the C oracle's
Crank-Nicolson F), then sweeps U^k_{n+1} = F(U^{k-1}_n) + (G(U^k_n) -
G(U^{k-1}_n)) for n = 0..N-1, with the defect max |U^k - U^{k-1}|.  Pure
Python loops over slices: small cases only.

Pins (tests/test_oracle_flowmap.py): finite termination (after N iterations
the iterate is the serial fine solution, bitwise, for any G, Sec. 3.1); a
network that ignores its first and third inputs reduces the flow-map coarse
to the state-independent network coarse of the C oracle; G is the network at
the stated inputs.
"""
from __future__ import annotations

import numpy as np

from . import fine, grid, initial
from .mlp import forward


def coarse(theta, depth, width, p, M, tau_s, tau_e, u):
    """G over one slice: K w(tau_s, tau_e, u_j / K, S_j / K) for every node."""
    S = grid(p, M)
    X = np.stack([np.full(M, tau_s), np.full(M, tau_e), np.asarray(u, float) / p.K, S / p.K], 1)
    return p.K * forward(theta, X, 4, depth, width)


def parareal(p, M, N, fine_steps, theta, depth, width, tol=0.0, max_iter=None, payoff_mode=1):
    """Flow-map Parareal.  Returns dict(U, iters, defects, iterates)."""
    max_iter = N if max_iter is None else max_iter
    dT = p.T / N
    U = np.empty((N + 1, M))
    U[0] = initial(p, M, payoff_mode)
    Gold = np.empty((N, M))
    for n in range(N):
        Gold[n] = coarse(theta, depth, width, p, M, n * dT, (n + 1) * dT, U[n])
        U[n + 1] = Gold[n]
    iterates = [U.copy()]
    defects = []
    k = 0
    while k < max_iter:
        k += 1
        Fv = np.stack([fine(p, M, n * dT, dT, fine_steps, U[n]) for n in range(N)])
        Unew = U.copy()
        for n in range(N):
            g = coarse(theta, depth, width, p, M, n * dT, (n + 1) * dT, Unew[n])
            Unew[n + 1] = Fv[n] + (g - Gold[n])
            Gold[n] = g
        defects.append(float(np.max(np.abs(Unew - U))))
        U = Unew
        iterates.append(U.copy())
        if defects[-1] <= tol or k == N:
            break
    return {"U": U, "iters": k, "defects": np.array(defects), "iterates": np.array(iterates)}
