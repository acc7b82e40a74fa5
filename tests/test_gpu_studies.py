"""GPU checks behind the studies (bench_studies.py) against the CPU oracle.

* Generalization (Sec. 4, Fig. 4): the network coarse is evaluated for one
  option while the fine and implicit-Euler steps use other r and sigma (up
  to 10 times the training values).  Every iterate of the network-coarse
  Parareal matches the oracle's on the same network grid normwise to 1e-12
  (the propagator tolerance), and iteration N is the serial fine solution.
* Data-only network (Sec. 4, Fig. 3): the loss of the value-matching set
  alone (n_f = n_b = 0, targets at arbitrary tau) and its gradient match the
  oracle's hand-written reverse mode (1e-4 relative, as for the residual
  loss); a short data-only training lowers the data misfit.
* Flow-map coarse (Sec. 3.3's interface read node by node): the coarse
  prediction against the oracle's FP64 flow-map Parareal (oracle/flowmap.py)
  within float32 rounding compounded over the slices (1e-4 normwise),
  iteration N equal to the serial fine solution (1e-12), the solve equal to
  the iteration path bitwise; a 2-input network is refused.
Weights and data are seeded draws; no GPU result feeds the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2303_03848_amd as bsp
from oracle import mlp
from paper_2303_03848_amd.pinn import DataLoss, train_on_data
from tests.gpu_util import cuda, normwise, say, to_dev
from workloads import SMALL_CALL, option_params, perturbed, xavier_normal

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which,factor", [("r", 10.0), ("sigma", 10.0), ("r", 0.5)])
@pytest.mark.parametrize("kind", [bsp.COARSE_PINN_IE, bsp.COARSE_PINN])
def test_network_coarse_at_other_parameters(which, factor, kind):
    cuda()
    cfg = dict(SMALL_CALL, r=0.03, sigma=0.4)
    p = option_params(cfg)
    p[which] = p[which] * factor
    M, N, Sf = cfg["M"], cfg["N"], cfg["fine_steps"]
    say(f"network coarse at {which} x {factor} kind={kind}")
    th = perturbed(xavier_normal(2, 4, 64, seed=5), 0.05, 6)
    net = bsp.PinnNet(to_dev(th, torch.float32), 2, 4, 64, bsp.PREC_FP32)
    po = oracle.params_from(p)
    taus = np.arange(N + 1) * (po.T / N)
    Vt = mlp.grid_values(th.astype(np.float64), 2, 4, 64, po.K, taus, oracle.grid(po, M))
    ref = oracle.parareal(po, M, N, Sf, 1, kind, Vt=Vt, tol=0.0)
    pr = bsp.Parareal(p, M, N, Sf, 1, kind, net)
    pr.start()
    for k in range(1, N + 1):
        pr.iterate(k)
    U = pr.U.cpu().numpy()
    assert normwise(U, ref["U"]) <= 1e-12
    ser = oracle.serial_fine(po, M, N, Sf)
    assert normwise(U, ser) <= 1e-12


def _data_points(n, seed=3):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(0.0, 1.0, n), rng.uniform(0.0, 3.0, n)], 1)
    y = np.maximum(X[:, 1] - 1.0, 0.0) + 0.1 * X[:, 0] + 0.01 * rng.normal(size=n)
    return X.astype(np.float32), y.astype(np.float32)


@pytest.mark.parametrize("depth,width,n", [(3, 32, 300), (4, 64, 1000), (2, 16, 1)])
def test_data_loss_matches_oracle(depth, width, n):
    cuda()
    th = perturbed(xavier_normal(2, depth, width, seed=7), 0.05, 8)
    X, y = _data_points(n)
    p = option_params(SMALL_CALL)
    spec = (2, depth, width, bsp.PREC_FP32)
    params = torch.nn.Parameter(to_dev(th, torch.float32))
    empty = torch.empty((0, 2), dtype=torch.float32, device="cuda")
    Xd, yd = to_dev(X, torch.float32), to_dev(y, torch.float32)
    loss = DataLoss.apply(params, spec, p, Xd, yd, empty, None)
    loss.backward()
    none = np.zeros((0, 2))
    f64 = lambda a: a.astype(np.float64)  # noqa: E731
    kw = dict(is_put=False, sigma=p["sigma"], r=p["r"], y_e=f64(y))
    rl3 = mlp.loss3(f64(th), none, f64(X), none, 2, depth, width, **kw)
    rg = mlp.loss_grad(f64(th), none, f64(X), none, 2, depth, width, **kw)
    assert rl3[0] == 0.0 and rl3[2] == 0.0
    np.testing.assert_allclose(float(loss), rl3[1], rtol=1e-4, atol=1e-9)
    g = params.grad.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(g - rg)) <= 1e-4 * np.max(np.abs(rg))


def test_train_on_data_lowers_misfit():
    cuda()
    X, y = _data_points(4096)
    p = option_params(SMALL_CALL)
    net0 = bsp.PinnNet(to_dev(xavier_normal(2, 3, 32, 0), torch.float32), 2, 3, 32,
                       bsp.PREC_FP32)
    v0 = bsp.pinn_forward(net0, to_dev(X, torch.float32)).cpu().numpy()
    net, info = train_on_data(p, X, y, 2, 3, 32, batch=1024, epochs_hi=40, epochs_lo=10)
    v = bsp.pinn_forward(net, to_dev(X, torch.float32)).cpu().numpy()
    mse0, mse = float(np.mean((v0 - y) ** 2)), float(np.mean((v - y) ** 2))
    say(f"data-only training: mse {mse0:.3e} -> {mse:.3e} ({info['steps']} steps)")
    assert info["steps"] == 50 * 4
    assert mse < 0.1 * mse0


@pytest.mark.parametrize("is_put,M", [(False, 256), (True, 256), (True, 5000)])
def test_flowmap_coarse_against_oracle(is_put, M):
    """The flow-map coarse (a 4-input network applied to the state node by
    node): the coarse prediction against the oracle's FP64 network within
    float32 rounding compounded over the slices, every later iterate ending
    in the serial fine solution (finite termination), and the solve's
    iterate equal to the iteration path's."""
    from oracle import flowmap
    cuda()
    cfg = dict(SMALL_CALL, is_put=is_put, M=M)
    if M > 4096:  # a grid for the large-grid fine kernel; fewer slices and steps
        cfg.update(N=4, fine_steps=6)
    p = option_params(cfg)
    N, Sf = cfg["N"], cfg["fine_steps"]
    say(f"flow-map coarse put={is_put} M={M}")
    th = perturbed(xavier_normal(4, 3, 32, seed=9), 0.05, 10)
    net = bsp.PinnNet(to_dev(th, torch.float32), 4, 3, 32, bsp.PREC_FP32)
    po = oracle.params_from(p)
    ref = flowmap.parareal(po, M, N, Sf, th.astype(np.float32).astype(np.float64), 3, 32, tol=0.0)
    pr = bsp.Parareal(p, M, N, Sf, 1, bsp.COARSE_FLOWMAP, net)
    U0 = pr.start().cpu().numpy()
    assert normwise(U0, ref["iterates"][0]) <= 1e-4
    d = [pr.iterate(k) for k in range(1, N + 1)]
    U = pr.U.cpu().numpy()
    # propagator bound (test_gpu_propagators.large_tol) on large grids
    dt = p["T"] / (N * Sf)
    bound = 1e-12 if M <= 4096 else max(
        1e-11, 16 * np.finfo(float).eps * N * Sf * (1 + dt * (p["sigma"] * M) ** 2))
    assert normwise(U, oracle.serial_fine(po, M, N, Sf)) <= bound
    assert np.all(np.isfinite(d)) and d[-1] < d[0]
    pr2 = bsp.Parareal(p, M, N, Sf, 1, bsp.COARSE_FLOWMAP, net)
    it, d2, rc = pr2.solve(0.0)
    assert it == N and rc == bsp.BS_OK
    assert np.array_equal(pr2.U.cpu().numpy(), U)
    assert d2 == d


def test_flowmap_refused_where_unsupported():
    cuda()
    p = option_params(SMALL_CALL)
    th = xavier_normal(2, 2, 16, seed=1)
    net = bsp.PinnNet(to_dev(th, torch.float32), 2, 2, 16, bsp.PREC_FP32)
    pr = bsp.Parareal(p, 64, 4, 8, 1, bsp.COARSE_FLOWMAP, net)
    with pytest.raises(bsp.BsError):
        pr.start()
    net4 = bsp.PinnNet(to_dev(xavier_normal(4, 2, 16, seed=1), torch.float32), 4, 2, 16,
                       bsp.PREC_FP32)
    with pytest.raises(bsp.BsError):
        bsp.parareal_solve_batch([dict(p, M=64, N=4, fine_steps=8, coarse_steps=1)],
                                 bsp.COARSE_FLOWMAP, 1e-8, net=net4)
