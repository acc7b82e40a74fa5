"""The FP64 network oracle against torch (a separate implementation):
forward values against a float64 nn.Sequential, the derivative streams
against torch.autograd.grad with create_graph, the PINN loss gradient against
torch autograd and against central finite differences.  The residual formula
is pinned on the closed-form price, whose residual vanishes."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from workloads import collocation, perturbed, xavier_normal


def _torch_net(theta, n_in, depth, width):
    layers, mods = mlp.unpack(theta, n_in, depth, width), []
    for W, b in layers[:-1]:
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        lin.weight.data = torch.tensor(W.copy())
        lin.bias.data = torch.tensor(b.copy())
        mods += [lin, torch.nn.Tanh()]
    W, b = layers[-1]
    lin = torch.nn.Linear(W.shape[1], 1).double()
    lin.weight.data = torch.tensor(W.copy())
    lin.bias.data = torch.tensor(b.copy())
    mods.append(lin)
    return torch.nn.Sequential(*mods)


def _torch_streams(net, X):
    Xt = torch.tensor(X, requires_grad=True)
    v = net(Xt)[:, 0]
    (g,) = torch.autograd.grad(v.sum(), Xt, create_graph=True)
    v_t, v_x = g[:, 0], g[:, 1]
    (gx,) = torch.autograd.grad(v_x.sum(), Xt, create_graph=True)
    return v, v_t, v_x, gx[:, 1]


CASES = [(2, 1, 5), (2, 3, 16), (2, 4, 64), (4, 4, 32)]


def _theta(n_in, depth, width):
    return perturbed(xavier_normal(n_in, depth, width, seed=width), 0.1, seed=depth).astype(np.float64)


@pytest.mark.parametrize("n_in,depth,width", CASES)
def test_forward_and_streams_vs_torch(n_in, depth, width):
    th = _theta(n_in, depth, width)
    box = ((0.1, 0.5), (0.0, 0.1)) if n_in == 4 else None
    X, _, _ = collocation(64, 1, 2, 1.0, 3.0, seed=5, coeff_box=box)
    net = _torch_net(th, n_in, depth, width)
    ref = [t.detach().numpy() for t in _torch_streams(net, X)]
    got = mlp.streams(th, X, n_in, depth, width)
    for g, r in zip(got, ref):
        assert np.max(np.abs(g - r)) <= 1e-13 * max(1.0, np.max(np.abs(r)))
    assert np.max(np.abs(mlp.forward(th, X, n_in, depth, width) - ref[0])) <= 1e-13


@pytest.mark.parametrize("n_in,depth,width", CASES)
@pytest.mark.parametrize("is_put", [False, True])
def test_loss_and_gradient_vs_torch_autograd(n_in, depth, width, is_put):
    th = _theta(n_in, depth, width)
    box = ((0.1, 0.5), (0.0, 0.1)) if n_in == 4 else None
    X_f, X_e, X_b = collocation(48, 16, 12, 1.0, 3.0, seed=6, coeff_box=box)
    sig, rr = (None, None) if n_in == 4 else (0.2, 0.05)
    net = _torch_net(th, n_in, depth, width)
    v, v_t, v_x, v_xx = _torch_streams(net, X_f)
    x = torch.tensor(X_f[:, 1])
    sg = torch.tensor(X_f[:, 2]) if n_in == 4 else sig
    rt = torch.tensor(X_f[:, 3]) if n_in == 4 else rr
    f = v_t - 0.5 * sg * sg * x * x * v_xx - rt * x * v_x + rt * v
    ve = net(torch.tensor(X_e))[:, 0]
    vb = net(torch.tensor(X_b))[:, 0]
    ye = torch.tensor(mlp.terminal_target(X_e, is_put))
    yb = torch.tensor(mlp.boundary_target(X_b, is_put, rr))
    terms = [(f * f).mean(), ((ve - ye) ** 2).mean(), ((vb - yb) ** 2).mean()]
    loss = terms[0] + terms[1] + terms[2]
    loss.backward()
    ref_grad = np.concatenate([torch.cat([m.weight.grad.reshape(-1), m.bias.grad]).numpy()
                               for m in net if isinstance(m, torch.nn.Linear)])
    got3 = mlp.loss3(th, X_f, X_e, X_b, n_in, depth, width, is_put, sig, rr)
    for g, r in zip(got3, terms):
        assert abs(g - r.item()) <= 1e-12 * max(1.0, abs(r.item()))
    got = mlp.loss_grad(th, X_f, X_e, X_b, n_in, depth, width, is_put, sig, rr)
    assert np.max(np.abs(got - ref_grad)) <= 1e-11 * max(1.0, np.max(np.abs(ref_grad)))


def test_gradient_vs_finite_differences():
    n_in, depth, width = 2, 3, 8
    th = _theta(n_in, depth, width)
    X_f, X_e, X_b = collocation(30, 10, 10, 1.0, 3.0, seed=7)
    g = mlp.loss_grad(th, X_f, X_e, X_b, n_in, depth, width, False, 0.2, 0.05)
    h = 1e-6
    fd = np.empty_like(th)
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = h
        fd[i] = (sum(mlp.loss3(th + e, X_f, X_e, X_b, n_in, depth, width, False, 0.2, 0.05))
                 - sum(mlp.loss3(th - e, X_f, X_e, X_b, n_in, depth, width, False, 0.2, 0.05))) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd))


@pytest.mark.parametrize("is_put", [False, True])
def test_residual_vanishes_on_closed_form(is_put):
    """The residual formula applied to the closed-form price (v = V/K,
    derivatives by central differences) is zero up to the differencing error."""
    K, r, sigma = 100.0, 0.05, 0.2
    x = np.linspace(0.5, 2.0, 7)
    tau, h = 0.6, 1e-4

    def v(t, xx):
        return oracle.bs_price(xx * K, K, r, sigma, t, is_put) / K

    v0 = v(tau, x)
    v_t = (v(tau + h, x) - v(tau - h, x)) / (2 * h)
    v_x = (v(tau, x + h) - v(tau, x - h)) / (2 * h)
    v_xx = (v(tau, x + h) - 2 * v0 + v(tau, x - h)) / h ** 2
    f = mlp.residual_from_streams(v0, v_t, v_x, v_xx, x, sigma, r)
    assert np.max(np.abs(f)) < 1e-5
    f_wrong = mlp.residual_from_streams(v0, -v_t, v_x, v_xx, x, sigma, r)
    assert np.max(np.abs(f_wrong)) > 1e-3


def test_targets():
    X = np.array([[0.0, 0.5], [0.0, 1.5]])
    assert np.allclose(mlp.terminal_target(X, False), [0.0, 0.5])
    assert np.allclose(mlp.terminal_target(X, True), [0.5, 0.0])
    Xb = np.array([[0.5, 0.0], [0.5, 3.0]])
    assert np.allclose(mlp.boundary_target(Xb, False, 0.05), [0.0, 3.0 - np.exp(-0.025)])
    assert np.allclose(mlp.boundary_target(Xb, True, 0.05), [np.exp(-0.025), 0.0])


def test_grid_values_layout():
    n_in, depth, width = 2, 2, 8
    th = _theta(n_in, depth, width)
    taus = np.array([0.0, 0.25, 1.0])
    S = np.array([10.0, 100.0, 250.0, 290.0])
    G = mlp.grid_values(th, n_in, depth, width, 100.0, taus, S)
    for i, t in enumerate(taus):
        for j, s in enumerate(S):
            ref = 100.0 * mlp.forward(th, np.array([[t, s / 100.0]]), n_in, depth, width)[0]
            assert G[i, j] == pytest.approx(ref, rel=1e-15, abs=1e-13)


def test_empty_point_sets_contribute_zero():
    n_in, depth, width = 2, 2, 8
    th = _theta(n_in, depth, width)
    X_f, X_e, X_b = collocation(20, 0, 6, 1.0, 3.0, seed=9)
    l3 = mlp.loss3(th, X_f, X_e, X_b, n_in, depth, width, False, 0.2, 0.05)
    assert l3[1] == 0.0 and np.isfinite(l3[0]) and np.isfinite(l3[2])
    g_empty = mlp.loss_grad(th, X_f, X_e, X_b, n_in, depth, width, False, 0.2, 0.05)
    g_none = mlp.loss_grad(th, X_f, X_e[:0], X_b, n_in, depth, width, False, 0.2, 0.05)
    assert np.array_equal(g_empty, g_none)


@pytest.mark.parametrize("n_f", [0, 40])
def test_value_targets_vs_torch_autograd(n_f):
    """Given value targets (y_e, y_b) replace eqs. (2)-(4): the loss and its
    gradient against torch autograd with the same targets; n_f = 0 is the loss
    of a network fitted to values alone (data, no residual)."""
    n_in, depth, width = 2, 3, 16
    th = _theta(n_in, depth, width)
    X_f, X_e, X_b = collocation(max(n_f, 1), 25, 10, 1.0, 3.0, seed=9)
    X_f = X_f[:n_f]
    rng = np.random.default_rng(4)
    y_e = rng.normal(size=X_e.shape[0])
    y_b = rng.normal(size=X_b.shape[0])
    net = _torch_net(th, n_in, depth, width)
    terms = []
    if n_f:
        v, v_t, v_x, v_xx = _torch_streams(net, X_f)
        x = torch.tensor(X_f[:, 1])
        f = v_t - 0.5 * 0.2 * 0.2 * x * x * v_xx - 0.05 * x * v_x + 0.05 * v
        terms.append((f * f).mean())
    else:
        terms.append(torch.zeros((), dtype=torch.float64))
    terms.append(((net(torch.tensor(X_e))[:, 0] - torch.tensor(y_e)) ** 2).mean())
    terms.append(((net(torch.tensor(X_b))[:, 0] - torch.tensor(y_b)) ** 2).mean())
    sum(terms).backward()
    ref_grad = np.concatenate([torch.cat([m.weight.grad.reshape(-1), m.bias.grad]).numpy()
                               for m in net if isinstance(m, torch.nn.Linear)])
    got3 = mlp.loss3(th, X_f, X_e, X_b, n_in, depth, width, False, 0.2, 0.05, y_e=y_e, y_b=y_b)
    for g, r in zip(got3, terms):
        assert abs(g - r.item()) <= 1e-12 * max(1.0, abs(r.item()))
    got = mlp.loss_grad(th, X_f, X_e, X_b, n_in, depth, width, False, 0.2, 0.05, y_e=y_e, y_b=y_b)
    assert np.max(np.abs(got - ref_grad)) <= 1e-11 * max(1.0, np.max(np.abs(ref_grad)))


def test_value_targets_equal_to_conditions_change_nothing():
    """Targets equal to eqs. (2)-(4) give the loss and gradient of the default."""
    n_in, depth, width = 2, 2, 8
    th = _theta(n_in, depth, width)
    X_f, X_e, X_b = collocation(20, 12, 8, 1.0, 3.0, seed=10)
    y_e = mlp.terminal_target(X_e, True)
    y_b = mlp.boundary_target(X_b, True, 0.05)
    a = mlp.loss3(th, X_f, X_e, X_b, n_in, depth, width, True, 0.2, 0.05)
    b = mlp.loss3(th, X_f, X_e, X_b, n_in, depth, width, True, 0.2, 0.05, y_e=y_e, y_b=y_b)
    assert a == b
    ga = mlp.loss_grad(th, X_f, X_e, X_b, n_in, depth, width, True, 0.2, 0.05)
    gb = mlp.loss_grad(th, X_f, X_e, X_b, n_in, depth, width, True, 0.2, 0.05, y_e=y_e, y_b=y_b)
    assert np.array_equal(ga, gb)


def test_bf16_round_vs_torch():
    """bf16_round against torch's float32 -> bfloat16 conversion, on spread
    values and on exact ties and their neighbours (ties go to even)."""
    rng = np.random.default_rng(3)
    x = (rng.normal(size=4000) * 10.0 ** rng.integers(-8, 8, size=4000)).astype(np.float32)
    u = rng.normal(size=2000).astype(np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    near = np.concatenate([u | np.uint32(0x8000), u | np.uint32(0x7FFF), u | np.uint32(0x8001),
                           u | np.uint32(0x18000)]).view(np.float32)
    for v in (x, near, np.array([0.0, -0.0, 1.0, -3.5], dtype=np.float32)):
        ref = torch.tensor(v).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(mlp.bf16_round(v), ref)
    assert np.array_equal(mlp.bf16_round(x.astype(np.float64)), mlp.bf16_round(x))


@pytest.mark.parametrize("n_in,depth,width", CASES)
def test_loss_grad_with_loss_matches_loss3(n_in, depth, width):
    th = _theta(n_in, depth, width)
    box = ((0.1, 0.5), (0.0, 0.1)) if n_in == 4 else None
    Xf, Xe, Xb = collocation(50, 9, 7, 1.0, 3.0, seed=4, coeff_box=box)
    kw = dict(is_put=True, sigma=None if n_in == 4 else 0.3, r=None if n_in == 4 else 0.04)
    l3 = mlp.loss3(th, Xf, Xe, Xb, n_in, depth, width, **kw)
    l, g = mlp.loss_grad(th, Xf, Xe, Xb, n_in, depth, width, with_loss=True, **kw)
    np.testing.assert_allclose(l, l3, rtol=1e-12, atol=1e-300)
    assert np.array_equal(g, mlp.loss_grad(th, Xf, Xe, Xb, n_in, depth, width, **kw))
    ident = mlp.loss_grad(th, Xf, Xe, Xb, n_in, depth, width, operand_round=lambda a: a, **kw)
    assert np.array_equal(g, ident)


def test_operand_rounding_only_in_hidden_products():
    """bf16 operand rounding touches the hidden-layer products only: a
    one-layer network (no such product) is unchanged bitwise; on a deeper one
    the value-set losses equal those of a float64 torch forward whose hidden
    products take operands rounded by torch's own bfloat16 conversion, and
    the gradient moves by no more than bfloat16 rounding allows."""
    Xf, Xe, Xb = collocation(40, 30, 20, 1.0, 3.0, seed=8)
    kw = dict(is_put=False, sigma=0.25, r=0.05)
    th1 = _theta(2, 1, 16)
    exact1 = mlp.loss_grad(th1, Xf, Xe, Xb, 2, 1, 16, with_loss=True, **kw)
    rnd1 = mlp.loss_grad(th1, Xf, Xe, Xb, 2, 1, 16, with_loss=True, operand_round=mlp.bf16_round,
                         **kw)
    assert exact1[0] == rnd1[0] and np.array_equal(exact1[1], rnd1[1])

    n_in, depth, width = 2, 3, 32
    th = _theta(n_in, depth, width)
    (l_r, g_r) = mlp.loss_grad(th, Xf, Xe, Xb, n_in, depth, width, with_loss=True,
                               operand_round=mlp.bf16_round, **kw)
    rt = lambda t: t.to(torch.float32).to(torch.bfloat16).to(torch.float64)  # noqa: E731
    layers = mlp.unpack(th, n_in, depth, width)

    def value(X):
        a = torch.tanh(torch.tensor(X) @ torch.tensor(layers[0][0]).T + torch.tensor(layers[0][1]))
        for W, b in layers[1:-1]:
            a = torch.tanh(rt(a) @ rt(torch.tensor(W)).T + torch.tensor(b))
        Wo, bo = layers[-1]
        return (a @ torch.tensor(Wo).T + torch.tensor(bo))[:, 0].numpy()

    ye, yb = mlp.terminal_target(Xe, False), mlp.boundary_target(Xb, False, 0.05)
    assert abs(l_r[1] - np.mean((value(Xe) - ye) ** 2)) <= 1e-13 * l_r[1]
    assert abs(l_r[2] - np.mean((value(Xb) - yb) ** 2)) <= 1e-13 * l_r[2]
    g = mlp.loss_grad(th, Xf, Xe, Xb, n_in, depth, width, **kw)
    dev = np.max(np.abs(g_r - g)) / np.max(np.abs(g))
    assert 0.0 < dev <= 5e-2
