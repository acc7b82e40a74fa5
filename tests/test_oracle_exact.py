"""Exact discrete solutions of the oracle's theta-method propagators.

Centred differences are exact on quadratics, so the semi-discrete operator L
of the paper's Sec. 3.2 satisfies, for S_j = j dS:
    L S = 0,   L 1 = -r,   L S^2 = (sigma^2 + r) S^2.
Hence, with Dirichlet data taken on the same discrete sequences, one theta
step of size dt maps
    S - K rho^m     -> S - K rho^{m+1},  rho = (1 - (1-theta) r dt) / (1 + theta r dt),
    S^2 mu^m        -> S^2 mu^{m+1},     mu = (1 + (1-theta) lam dt) / (1 - theta lam dt),
with lam = sigma^2 + r.  A wrong sign, a dropped factor 1/2 or a misplaced
boundary term in the operator, the step or the boundary handling breaks one
of these identities.  theta = 1/2 is Crank-Nicolson (fine F), theta = 1 is
implicit Euler (coarse G).
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("theta", [0.5, 1.0])
@pytest.mark.parametrize("M", [1, 7, 64, 256])
def test_affine_solution(theta, M):
    p = oracle.params(100.0, 0.05, 0.2, 1.0, 300.0)
    dt, steps = 0.013, 40
    rho = (1 - (1 - theta) * p.r * dt) / (1 + theta * p.r * dt)
    m = np.arange(steps + 1)
    g_lo = 0.0 - p.K * rho ** m
    g_hi = p.s_max - p.K * rho ** m
    S = oracle.grid(p, M)
    out = oracle.propagate_bc(p, M, theta, dt, steps, g_lo, g_hi, S - p.K)
    exact = S - p.K * rho ** steps
    assert np.max(np.abs(out - exact)) <= 1e-12 * p.s_max


@pytest.mark.parametrize("theta", [0.5, 1.0])
@pytest.mark.parametrize("sigma,r", [(0.2, 0.05), (0.5, 0.0), (0.1, 0.1)])
def test_quadratic_solution(theta, sigma, r):
    M = 200
    p = oracle.params(100.0, r, sigma, 1.0, 300.0)
    lam = sigma ** 2 + r
    dt, steps = 0.02, 30
    mu = (1 + (1 - theta) * lam * dt) / (1 - theta * lam * dt)
    m = np.arange(steps + 1)
    g_lo = np.zeros(steps + 1)
    g_hi = p.s_max * mu ** m
    S = oracle.grid(p, M)
    out = oracle.propagate_bc(p, M, theta, dt, steps, g_lo, g_hi, S * S / p.s_max)
    exact = S * S / p.s_max * mu ** steps
    assert np.max(np.abs(out - exact)) <= 1e-13 * np.max(np.abs(exact))


def test_theta_step_orders():
    """theta = 1/2 is second order in time, theta = 1 first order: on the
    eigen-solution S^2 the one-step growth factor matches exp(lam dt) to
    O(dt^3) and O(dt^2) respectively."""
    lam, dt = 0.09, 0.05
    cn = (1 + 0.5 * lam * dt) / (1 - 0.5 * lam * dt)
    ie = 1 / (1 - lam * dt)
    assert abs(cn - np.exp(lam * dt)) < (lam * dt) ** 3
    assert abs(ie - np.exp(lam * dt)) < (lam * dt) ** 2
