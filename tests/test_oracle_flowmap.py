"""Pins of the oracle's flow-map Parareal (oracle/flowmap.py; Sec. 3.1 eq. (7)
with the coarse interface of Sec. 3.3 read node by node).

* Finite termination (Sec. 3.1): whatever the coarse propagator, after k
  iterations the slices n <= k hold the serial fine solution bitwise, and
  after N iterations the whole iterate does.
* A network whose weights ignore the slice start and the state (first and
  third inputs) is a function of (tau_end, S/K) alone: the flow-map coarse
  is then the state-independent network coarse, so the iterates equal the
  C oracle's Parareal with the literal network kind on that network's grid.
* The coarse propagator is the network at (tau_s, tau_e, u/K, S/K) times K.
"""
import numpy as np

import oracle
from oracle import flowmap, mlp
from workloads import SMALL_CALL, option_params, perturbed, xavier_normal

CFG = dict(SMALL_CALL, N=6, fine_steps=16, M=96)


def _p():
    return oracle.params_from(option_params(CFG))


def _theta(depth=3, width=16, seed=2):
    return perturbed(xavier_normal(4, depth, width, seed=seed), 0.05, seed + 1).astype(np.float64)


def test_finite_termination_and_front():
    p, M, N = _p(), CFG["M"], CFG["N"]
    r = flowmap.parareal(p, M, N, CFG["fine_steps"], _theta(), 3, 16, tol=0.0)
    ser = oracle.serial_fine(p, M, N, CFG["fine_steps"])
    assert r["iters"] == N
    assert np.array_equal(r["U"], ser)
    for k in range(1, N + 1):
        assert np.array_equal(r["iterates"][k][: k + 1], ser[: k + 1]), k
    # the prediction is not the fine solution (the pin above is not vacuous)
    assert np.abs(r["iterates"][0][N] - ser[N]).max() > 1e-3


def test_state_blind_network_is_the_literal_network_coarse():
    p, M, N = _p(), CFG["M"], CFG["N"]
    depth, width = 3, 16
    th4 = _theta(depth, width)
    W1 = th4[: 4 * width].reshape(width, 4).copy()
    W1[:, 0] = 0.0  # slice start
    W1[:, 2] = 0.0  # state
    th4[: 4 * width] = W1.ravel()
    # the same network on (tau, S/K): the first layer's columns 1 and 3
    th2 = np.concatenate([W1[:, [1, 3]].ravel(), th4[4 * width:]])
    taus = np.arange(N + 1) * (p.T / N)
    Vt = mlp.grid_values(th2, 2, depth, width, p.K, taus, oracle.grid(p, M))
    a = flowmap.parareal(p, M, N, CFG["fine_steps"], th4, depth, width, tol=0.0)
    b = oracle.parareal(p, M, N, CFG["fine_steps"], 1, oracle.COARSE_PINN, Vt=Vt, tol=0.0,
                        keep_iterates=True)
    scale = np.abs(b["iterates"]).max()
    assert np.abs(a["iterates"] - b["iterates"]).max() <= 1e-14 * scale


def test_coarse_is_the_network_at_the_slice_inputs():
    p, M = _p(), CFG["M"]
    th = _theta()
    u = np.linspace(0.0, 200.0, M)
    S = oracle.grid(p, M)
    g = flowmap.coarse(th, 3, 16, p, M, 0.25, 0.5, u)
    for j in (0, M // 3, M - 1):
        x = np.array([[0.25, 0.5, u[j] / p.K, S[j] / p.K]])
        # one row against the batch: the same sums up to their order
        assert abs(g[j] - p.K * mlp.forward(th, x, 4, 3, 16)[0]) <= 1e-13 * p.K
