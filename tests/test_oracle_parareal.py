"""Invariants of the oracle's Parareal iteration (paper Sec. 3.1, eq. (7)).

* N = 1: one iteration reproduces F.
* G := F (coarse Crank-Nicolson with the fine step count): the coarse
  prediction is already the serial fine solution, so the first defect is 0.
* Finite termination (Sec. 3.1: the iterates converge to the serial fine
  solution as k -> N): after k iterations the slices n <= k agree with serial
  fine integration bitwise, and after N iterations the whole iterate does.
* The state-independent network coarse collapses eq. (7) to U^k_{n+1} =
  F(U^{k-1}_n) (its G terms cancel exactly).
* The network-anchored coarse with an exact network gives a coarse
  prediction equal to the serial fine solution, so the first defect is 0.
* The numerical coarse propagator converges to tol before k = N on the
  network workload's grid.
* With the anchor set to the numerical coarse trajectory itself, the
  network-anchored coarse (anchor + implicit Euler with zero boundary data
  on the deviation) equals the numerical coarse, by linearity of the
  implicit-Euler map, for any number of coarse steps per slice: this pins
  the deviation solve's step size and step count.
"""
import numpy as np
import pytest

import oracle
from workloads import SMALL_CALL, option_params


def _p(cfg):
    return oracle.params_from(option_params(cfg))


def test_single_slice_equals_fine():
    cfg = SMALL_CALL
    p = _p(cfg)
    r = oracle.parareal(p, cfg["M"], 1, 64, 1, oracle.COARSE_IE, tol=0.0)
    U0 = oracle.initial(p, cfg["M"])
    F = oracle.fine(p, cfg["M"], 0.0, p.T, 64, U0)
    assert r["iters"] == 1
    assert np.array_equal(r["U"][1], F)


def test_coarse_equal_fine_converges_at_once():
    cfg = SMALL_CALL
    p = _p(cfg)
    r = oracle.parareal(p, cfg["M"], cfg["N"], cfg["fine_steps"], cfg["fine_steps"],
                        oracle.COARSE_CN, tol=0.0, max_iter=2)
    assert r["defects"][0] == 0.0


@pytest.mark.parametrize("kind", [oracle.COARSE_IE, oracle.COARSE_PINN, oracle.COARSE_PINN_IE])
def test_finite_termination_and_front(kind):
    cfg = SMALL_CALL
    p = _p(cfg)
    M, N = cfg["M"], cfg["N"]
    ser = oracle.serial_fine(p, M, N, cfg["fine_steps"])
    Vt = None
    if kind != oracle.COARSE_IE:
        # any prediction will do for the invariants: a perturbed closed form
        S = oracle.grid(p, M)
        taus = np.linspace(0, p.T, N + 1)
        Vt = np.stack([oracle.bs_price(S, p.K, p.r, p.sigma, t) for t in taus])
        Vt = Vt * (1 + 1e-2 * np.sin(S / 7.0))[None, :]
    r = oracle.parareal(p, M, N, cfg["fine_steps"], 1, kind, Vt=Vt, tol=0.0, keep_iterates=True)
    assert r["iters"] == N
    assert np.array_equal(r["U"], ser)
    for k, Uk in enumerate(r["iterates"]):
        assert np.array_equal(Uk[: k + 1], ser[: k + 1]), k


def test_literal_network_coarse_collapses_to_fine_sweep():
    cfg = SMALL_CALL
    p = _p(cfg)
    M, N = cfg["M"], cfg["N"]
    S = oracle.grid(p, M)
    taus = np.linspace(0, p.T, N + 1)
    Vt = np.stack([oracle.bs_price(S, p.K, p.r, p.sigma, t) for t in taus])
    r = oracle.parareal(p, M, N, cfg["fine_steps"], 1, oracle.COARSE_PINN, Vt=Vt, tol=0.0,
                        keep_iterates=True)
    its = r["iterates"]
    dT = p.T / N
    for k in range(1, 4):
        for n in range(N):
            Fv = oracle.fine(p, M, n * dT, dT, cfg["fine_steps"], its[k - 1][n])
            assert np.array_equal(its[k][n + 1], Fv)


def test_exact_network_anchor_gives_zero_first_defect():
    cfg = SMALL_CALL
    p = _p(cfg)
    M, N = cfg["M"], cfg["N"]
    ser = oracle.serial_fine(p, M, N, cfg["fine_steps"])
    r = oracle.parareal(p, M, N, cfg["fine_steps"], 1, oracle.COARSE_PINN_IE, Vt=ser, tol=0.0,
                        max_iter=1)
    assert r["defects"][0] == 0.0
    assert np.array_equal(r["U"], ser)


def test_numeric_coarse_defects_decrease_and_converge():
    cfg = dict(SMALL_CALL, M=256, N=32, fine_steps=32)
    p = _p(cfg)
    r = oracle.parareal(p, cfg["M"], cfg["N"], cfg["fine_steps"], 1, oracle.COARSE_IE,
                        tol=1e-8)
    d = r["defects"]
    assert r["status"] == 0 and r["iters"] < cfg["N"]
    assert d[-1] <= 1e-8
    assert np.all(d[1:] < d[:-1])
    ser = oracle.serial_fine(p, cfg["M"], cfg["N"], cfg["fine_steps"])
    assert np.max(np.abs(r["U"] - ser)) <= 1e-8


def test_threads_do_not_change_result():
    cfg = SMALL_CALL
    p = _p(cfg)
    a = oracle.parareal(p, cfg["M"], cfg["N"], cfg["fine_steps"], 1, oracle.COARSE_IE, tol=1e-8,
                        nthreads=1)
    b = oracle.parareal(p, cfg["M"], cfg["N"], cfg["fine_steps"], 1, oracle.COARSE_IE, tol=1e-8,
                        nthreads=4)
    assert np.array_equal(a["U"], b["U"]) and a["iters"] == b["iters"]


@pytest.mark.parametrize("coarse_steps", [1, 3])
def test_network_anchor_on_coarse_trajectory_equals_numeric_coarse(coarse_steps):
    cfg = dict(SMALL_CALL, N=6, fine_steps=16)
    p = _p(cfg)
    M, N = cfg["M"], cfg["N"]
    dT = p.T / N
    Vt = np.empty((N + 1, M))
    Vt[0] = oracle.initial(p, M)
    for n in range(N):
        Vt[n + 1] = oracle.coarse_ie(p, M, n * dT, dT, coarse_steps, Vt[n])
    a = oracle.parareal(p, M, N, cfg["fine_steps"], coarse_steps, oracle.COARSE_PINN_IE, Vt=Vt,
                        tol=0.0, keep_iterates=True)
    b = oracle.parareal(p, M, N, cfg["fine_steps"], coarse_steps, oracle.COARSE_IE, tol=0.0,
                        keep_iterates=True)
    scale = np.abs(b["iterates"]).max()
    assert np.abs(a["iterates"] - b["iterates"]).max() <= 1e-12 * scale
    # a wrong step (the whole slice in each of the coarse steps) breaks it
    if coarse_steps > 1:
        wrong = np.empty_like(Vt)
        wrong[0] = Vt[0]
        for n in range(N):
            wrong[n + 1] = oracle.coarse_ie(p, M, n * dT, coarse_steps * dT, coarse_steps,
                                            wrong[n])
        c = oracle.parareal(p, M, N, cfg["fine_steps"], coarse_steps, oracle.COARSE_PINN_IE,
                            Vt=wrong, tol=0.0, keep_iterates=True)
        assert np.abs(c["iterates"][0] - b["iterates"][0]).max() > 1e-6 * scale
