"""GPU network kernels against the FP64 oracle network (oracle/mlp.py).

* pinn_forward, float32: |v_gpu - v_ora| <= 2e-5 (1 + |v|): float32 rounding
  of at most 256-term dot products through <= 6 tanh layers.
* pinn_forward, bfloat16 operands / float32 accumulation: the error against
  the FP64 network is reported per case and bounded by 5e-2 (1 + |v|): bf16
  keeps 8 mantissa bits, ~4e-3 relative per layer.
* pinn_residual_fwd_bwd, float32: the three loss terms to 1e-4 relative and
  the gradient normwise to 1e-4 of its max (float32 sums over up to 9e3
  points and 4 streams), plus a directional finite difference of the GPU loss.
* bfloat16 residual path (one fused launch): against the oracle with the
  hidden-layer products on bfloat16-rounded operands, loss terms and gradient
  to 1e-3 (the derivation is at BF16_TOL); bitwise reproducible.
Weights are seeded draws; no GPU result feeds the oracle.
"""
import numpy as np
import pytest
import torch

import paper_2303_03848_amd as bsp
from oracle import mlp
from paper_2303_03848_amd.pinn import PinnResidualLoss
from tests.gpu_util import cuda, say, to_dev
from workloads import TRAIN_STEP, collocation, option_params, perturbed, xavier_normal

pytestmark = pytest.mark.gpu

CALL = option_params(TRAIN_STEP)


def _theta(n_in, depth, width, seed=0, noise=0.05):
    return perturbed(xavier_normal(n_in, depth, width, seed=seed), noise, seed + 1)


def _points(n_f, n_e, n_b, n_in, seed=11):
    box = ((0.1, 0.5), (0.0, 0.1)) if n_in == 4 else None
    return collocation(n_f, n_e, n_b, 1.0, 3.0, seed=seed, coeff_box=box)


@pytest.mark.parametrize("n_in,depth,width", [(2, 1, 16), (2, 4, 64), (2, 3, 128), (4, 4, 128),
                                              (2, 6, 256), (4, 2, 32)])
@pytest.mark.parametrize("n", [1, 33, 1000])
def test_forward_fp32(n_in, depth, width, n):
    cuda()
    th = _theta(n_in, depth, width)
    X, _, _ = _points(n, 1, 2, n_in)
    net = bsp.PinnNet(to_dev(th, torch.float32), n_in, depth, width, bsp.PREC_FP32)
    got = bsp.pinn_forward(net, to_dev(X, torch.float32)).cpu().numpy()
    ref = mlp.forward(th.astype(np.float64), X.astype(np.float32).astype(np.float64), n_in, depth,
                      width)
    assert np.max(np.abs(got - ref) / (1 + np.abs(ref))) <= 2e-5


@pytest.mark.parametrize("n_in,depth,width", [(2, 4, 64), (2, 4, 128), (4, 4, 128), (2, 6, 256),
                                              (2, 2, 32)])
def test_forward_bf16(n_in, depth, width):
    cuda()
    th = _theta(n_in, depth, width)
    X, _, _ = _points(1000, 1, 2, n_in)
    net = bsp.PinnNet(to_dev(th, torch.float32), n_in, depth, width, bsp.PREC_BF16)
    got = bsp.pinn_forward(net, to_dev(X, torch.float32)).cpu().numpy()
    ref = mlp.forward(th.astype(np.float64), X.astype(np.float32).astype(np.float64), n_in, depth,
                      width)
    err = np.max(np.abs(got - ref) / (1 + np.abs(ref)))
    say(f"bf16 forward {n_in}x{depth}x{width}: max |dv|/(1+|v|) = {err:.3e}")
    assert err <= 5e-2


def _gpu_loss(th, spec, p, Xf, Xe, Xb):
    net = bsp.PinnNet(to_dev(th, torch.float32), *spec)
    l3, g = bsp.pinn_residual_fwd_bwd(net, p, to_dev(Xf, torch.float32), to_dev(Xe, torch.float32),
                                      to_dev(Xb, torch.float32))
    return l3.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)


def _ora(th, n_in, depth, width, Xf, Xe, Xb, is_put):
    # the oracle sees exactly the float32 inputs the GPU sees
    f32 = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    t = th.astype(np.float64)
    kw = dict(is_put=is_put, sigma=None if n_in == 4 else CALL["sigma"],
              r=None if n_in == 4 else CALL["r"])
    l3 = np.array(mlp.loss3(t, f32(Xf), f32(Xe), f32(Xb), n_in, depth, width, **kw))
    g = mlp.loss_grad(t, f32(Xf), f32(Xe), f32(Xb), n_in, depth, width, **kw)
    return l3, g


CASES = [(2, 3, 32, 300, 40, 20), (2, 4, 64, 1000, 100, 33), (4, 4, 32, 257, 31, 17),
         (2, 2, 128, 640, 64, 64), (2, 4, 16, 100, 0, 10), (2, 1, 64, 50, 7, 0)]


@pytest.mark.parametrize("is_put", [False, True])
@pytest.mark.parametrize("n_in,depth,width,nf,ne,nb", CASES)
def test_residual_fp32(n_in, depth, width, nf, ne, nb, is_put):
    cuda()
    th = _theta(n_in, depth, width)
    Xf, Xe, Xb = _points(nf, ne, nb, n_in)
    p = dict(CALL, is_put=is_put)
    l3, g = _gpu_loss(th, (n_in, depth, width, bsp.PREC_FP32), p, Xf, Xe, Xb)
    rl3, rg = _ora(th, n_in, depth, width, Xf, Xe, Xb, is_put)
    np.testing.assert_allclose(l3, rl3, rtol=1e-4, atol=1e-9)
    assert np.max(np.abs(g - rg)) <= 1e-4 * np.max(np.abs(rg))


def test_residual_fp32_directional_fd():
    cuda()
    n_in, depth, width = 2, 3, 32
    th = _theta(n_in, depth, width).astype(np.float64)
    Xf, Xe, Xb = _points(400, 50, 30, n_in)
    spec = (n_in, depth, width, bsp.PREC_FP32)
    _, g = _gpu_loss(th, spec, CALL, Xf, Xe, Xb)
    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.normal(size=th.size)
        d /= np.linalg.norm(d)
        h = 1e-2
        lp, _ = _gpu_loss(th + h * d, spec, CALL, Xf, Xe, Xb)
        lm, _ = _gpu_loss(th - h * d, spec, CALL, Xf, Xe, Xb)
        fd = (lp.sum() - lm.sum()) / (2 * h)
        assert abs(fd - g @ d) <= 1e-3 * max(abs(fd), np.abs(g).max() * 1e-2)


def test_residual_full_training_batch():
    """The training-step workload at full size: 8192 interior, 512 terminal,
    256 boundary points, 128 x 4 network, float32, against the FP64 oracle."""
    cuda()
    c = TRAIN_STEP
    th = _theta(c["n_in"], c["depth"], c["width"])
    Xf, Xe, Xb = collocation(c["batch_f"], c["batch_e"], c["batch_b"], c["T"], c["s_max"] / c["K"])
    l3, g = _gpu_loss(th, (c["n_in"], c["depth"], c["width"], bsp.PREC_FP32), CALL, Xf, Xe, Xb)
    rl3, rg = _ora(th, c["n_in"], c["depth"], c["width"], Xf, Xe, Xb, False)
    np.testing.assert_allclose(l3, rl3, rtol=1e-4)
    assert np.max(np.abs(g - rg)) <= 1e-4 * np.max(np.abs(rg))


def _ora_bf16(th, n_in, depth, width, Xf, Xe, Xb, is_put):
    """The oracle with the hidden-layer products on bfloat16-rounded operands
    (the arithmetic of the matrix-core pass), everything else FP64."""
    f32 = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    kw = dict(is_put=is_put, sigma=None if n_in == 4 else CALL["sigma"],
              r=None if n_in == 4 else CALL["r"])
    l3, g = mlp.loss_grad(f32(th), f32(Xf), f32(Xe), f32(Xb), n_in, depth, width,
                          operand_round=mlp.bf16_round, with_loss=True, **kw)
    return np.array(l3), g


# Tolerance of the bfloat16 pass against the bfloat16-operand oracle: both
# round the same operands, so what remains is float32 arithmetic (about 1e-6
# relative) and the rare operand whose float32 value lies on the other side
# of a bfloat16 rounding boundary than the oracle's (one bfloat16 step,
# 4e-3, in one term of a sum of >= 32): 1e-3 leaves a margin of ten or more.
BF16_TOL = 1e-3

BF16_CASES = [(2, 4, 64, 1000, 100, 50), (2, 4, 128, 1000, 100, 50), (4, 4, 128, 257, 31, 17),
              (2, 3, 32, 1000, 100, 50), (2, 1, 64, 50, 7, 0), (2, 2, 32, 1, 0, 0),
              (2, 2, 64, 0, 40, 9), (2, 4, 128, 20000, 600, 300), (2, 6, 64, 700, 50, 30),
              (4, 5, 128, 300, 20, 20), (2, 3, 128, 33, 1, 1)]


@pytest.mark.parametrize("n_in,depth,width,nf,ne,nb", BF16_CASES)
def test_residual_bf16(n_in, depth, width, nf, ne, nb):
    """The fused bfloat16 step: single points, empty sets, ragged tiles, one
    hidden layer or none, 654 tiles (three per block), and networks of 5 and
    6 layers (the kernel with the caches in the point-major workspace)."""
    cuda()
    th = _theta(n_in, depth, width)
    Xf, Xe, Xb = _points(nf, ne, nb, n_in)
    say(f"bf16 residual {n_in}x{depth}x{width} points {nf}/{ne}/{nb}")
    l3, g = _gpu_loss(th, (n_in, depth, width, bsp.PREC_BF16), CALL, Xf, Xe, Xb)
    rl3, rg = _ora_bf16(th, n_in, depth, width, Xf, Xe, Xb, False)
    el = np.max(np.abs(l3 - rl3) / np.maximum(np.abs(rl3), 1e-30))
    eg = np.max(np.abs(g - rg)) / np.max(np.abs(rg))
    xl3, xg = _ora(th, n_in, depth, width, Xf, Xe, Xb, False)
    say(f"  vs bf16-operand oracle: loss {el:.2e}, grad {eg:.2e}; vs exact: grad "
        f"{np.max(np.abs(g - xg)) / np.max(np.abs(xg)):.2e}")
    assert np.all(l3[rl3 == 0.0] == 0.0)
    assert el <= BF16_TOL and eg <= BF16_TOL


@pytest.mark.parametrize("depth", [4, 6])
def test_residual_bf16_value_targets(depth):
    """Given value targets on the terminal and boundary sets (both bfloat16
    kernels: 4 and 6 layers), against the bfloat16-operand oracle."""
    cuda()
    th = _theta(2, depth, 64)
    Xf, Xe, Xb = _points(500, 70, 45, 2)
    rng = np.random.default_rng(21)
    ye = rng.normal(0.2, 0.1, Xe.shape[0]).astype(np.float32)
    yb = rng.normal(0.1, 0.1, Xb.shape[0]).astype(np.float32)
    net = bsp.PinnNet(to_dev(th, torch.float32), 2, depth, 64, bsp.PREC_BF16)
    l3, g = bsp.pinn_residual_fwd_bwd(net, CALL, to_dev(Xf, torch.float32),
                                      to_dev(Xe, torch.float32), to_dev(Xb, torch.float32),
                                      y_e=to_dev(ye, torch.float32), y_b=to_dev(yb, torch.float32))
    l3, g = l3.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    rl3, rg = mlp.loss_grad(f32(th), f32(Xf), f32(Xe), f32(Xb), 2, depth, 64, is_put=False,
                            sigma=CALL["sigma"], r=CALL["r"], y_e=f32(ye), y_b=f32(yb),
                            operand_round=mlp.bf16_round, with_loss=True)
    el = np.max(np.abs(l3 - np.array(rl3)) / np.abs(np.array(rl3)))
    eg = np.max(np.abs(g - rg)) / np.max(np.abs(rg))
    say(f"bf16 residual with value targets, {depth} layers: loss {el:.2e}, grad {eg:.2e}")
    assert el <= BF16_TOL and eg <= BF16_TOL


def test_residual_bf16_full_training_batch():
    """The training-step workload at full size in bfloat16 (8192 / 512 / 256
    points, 128 x 4) against the bfloat16-operand oracle, and bitwise
    reproducible from call to call."""
    cuda()
    c = TRAIN_STEP
    th = _theta(c["n_in"], c["depth"], c["width"])
    Xf, Xe, Xb = collocation(c["batch_f"], c["batch_e"], c["batch_b"], c["T"], c["s_max"] / c["K"])
    spec = (c["n_in"], c["depth"], c["width"], bsp.PREC_BF16)
    l3, g = _gpu_loss(th, spec, CALL, Xf, Xe, Xb)
    l3b, gb = _gpu_loss(th, spec, CALL, Xf, Xe, Xb)
    assert np.array_equal(l3, l3b) and np.array_equal(g, gb)
    rl3, rg = _ora_bf16(th, c["n_in"], c["depth"], c["width"], Xf, Xe, Xb, False)
    el = np.max(np.abs(l3 - rl3) / np.abs(rl3))
    eg = np.max(np.abs(g - rg)) / np.max(np.abs(rg))
    say(f"bf16 training batch: loss {el:.2e}, grad {eg:.2e}")
    assert el <= BF16_TOL and eg <= BF16_TOL


def test_autograd_function_and_adam_steps():
    cuda()
    n_in, depth, width = 2, 3, 32
    th = _theta(n_in, depth, width)
    Xf, Xe, Xb = (to_dev(a, torch.float32) for a in _points(512, 64, 32, n_in))
    params = torch.nn.Parameter(to_dev(th, torch.float32))
    spec = (n_in, depth, width, bsp.PREC_FP32)
    loss = PinnResidualLoss.apply(params, spec, CALL, Xf, Xe, Xb, None)
    loss.backward()
    _, g = bsp.pinn_residual_fwd_bwd(bsp.PinnNet(params.data, *spec), CALL, Xf, Xe, Xb)
    assert torch.equal(params.grad, g)
    opt = torch.optim.Adam([params], lr=1e-2)
    first = float(loss.detach())
    for _ in range(30):
        opt.zero_grad()
        loss = PinnResidualLoss.apply(params, spec, CALL, Xf, Xe, Xb, None)
        loss.backward()
        opt.step()
    assert float(loss) < first
