"""Training the physics-informed network (paper Sec. 3.3) through the
hand-written loss-and-gradient kernel.

``PinnResidualLoss`` is a ``torch.autograd.Function``: its forward calls
``pinn_residual_fwd_bwd`` (one pass computing the three loss terms of
eqs. (12)-(14) and the gradient of their sum, eq. (11)); its backward returns
that gradient scaled by the incoming gradient.  torch provides only the
optimiser (Adam, as in the paper) and device memory.

Training recipe (Sec. 3.3): fixed sets of uniformly drawn collocation points
(interior, terminal, boundary), reshuffled every epoch and taken in
minibatches (an epoch is one pass over the sets: 8 minibatches of 8192 / 512 /
256 points for the default sets); Adam with a learning rate of 1e-2, then
1e-3, for the paper's 5000 + 800 epochs by default.
"""
from __future__ import annotations

import time

import numpy as np
import torch

import paper_2303_03848_amd as bsp
from workloads import SEED, collocation, minibatch_indices, option_params, xavier_normal


class PinnResidualLoss(torch.autograd.Function):
    """total = MSE_f + MSE_exp + MSE_b as a differentiable function of the flat parameters."""

    @staticmethod
    def forward(ctx, params, spec, p, X_f, X_e, X_b, ws):
        net = bsp.PinnNet(params.detach(), *spec)
        loss3, grad = bsp.pinn_residual_fwd_bwd(net, p, X_f, X_e, X_b, ws=ws)
        ctx.save_for_backward(grad)
        ctx.loss3 = loss3
        return loss3.sum()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None, None, None


class DataLoss(torch.autograd.Function):
    """Mean squared error between the network and value targets (the
    residual kernel's value-matching set alone); loss and gradient in one
    pass of the kernel."""

    @staticmethod
    def forward(ctx, params, spec, p, X, y, empty, ws):
        net = bsp.PinnNet(params.detach(), *spec)
        loss3, grad = bsp.pinn_residual_fwd_bwd(net, p, empty, X, empty, ws=ws, y_e=y)
        ctx.save_for_backward(grad)
        return loss3[1].clone()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None, None, None


def pinn_loss(params: torch.Tensor, spec, p: dict, X_f, X_e, X_b, ws=None):
    """(total loss [differentiable w.r.t. params], loss3 [detached])."""
    total = PinnResidualLoss.apply(params, spec, p, X_f, X_e, X_b, ws)
    return total


def train(p: dict, n_in: int, depth: int, width: int, precision: int = bsp.PREC_FP32,
          n_f: int = 65536, n_e: int = 4096, n_b: int = 2048, batch=(8192, 512, 256),
          epochs_hi: int = 5000, epochs_lo: int = 800, lr_hi: float = 1e-2, lr_lo: float = 1e-3,
          seed: int = SEED, init_seed: int = 0, coeff_box=None, log_every: int = 0):
    """Train a network on the option `p` (or, with coeff_box, on a box of
    (sigma, r)) for epochs_hi epochs at lr_hi, then epochs_lo at lr_lo;
    returns (PinnNet, info dict)."""
    dev = torch.device("cuda")
    x_max = p["s_max"] / p["K"]
    Xf, Xe, Xb = collocation(n_f, n_e, n_b, p["T"], x_max, seed=seed, coeff_box=coeff_box)
    Xf, Xe, Xb = (torch.tensor(a, dtype=torch.float32, device=dev) for a in (Xf, Xe, Xb))
    params = torch.nn.Parameter(torch.tensor(xavier_normal(n_in, depth, width, init_seed),
                                             device=dev))
    spec = (n_in, depth, width, precision)
    net = bsp.PinnNet(params.data, *spec)
    ws = torch.empty(bsp.pinn_residual_workspace_size(net, *batch), dtype=torch.uint8, device=dev)
    opt = torch.optim.Adam([params], lr=lr_hi)
    nb_f, nb_e, nb_b = batch
    per_epoch = min(n_f // nb_f, n_e // nb_e, n_b // nb_b)
    steps_hi = epochs_hi * per_epoch
    total_steps = (epochs_hi + epochs_lo) * per_epoch
    t0 = time.time()
    step, epoch, hist = 0, 0, []
    while step < total_steps:
        idx_f = minibatch_indices(n_f, nb_f, epoch, seed)
        idx_e = minibatch_indices(n_e, nb_e, epoch, seed + 1)
        idx_b = minibatch_indices(n_b, nb_b, epoch, seed + 2)
        for q in range(per_epoch):
            if step == steps_hi:
                for gopt in opt.param_groups:
                    gopt["lr"] = lr_lo
            fi = torch.as_tensor(idx_f[q], device=dev)
            ei = torch.as_tensor(idx_e[q], device=dev)
            bi = torch.as_tensor(idx_b[q], device=dev)
            opt.zero_grad(set_to_none=True)
            loss = PinnResidualLoss.apply(params, spec, p, Xf[fi].contiguous(),
                                          Xe[ei].contiguous(), Xb[bi].contiguous(), ws)
            loss.backward()
            opt.step()
            step += 1
            if log_every and step % log_every == 0:
                hist.append((step, float(loss.detach())))
            if step >= total_steps:
                break
        epoch += 1
    torch.cuda.synchronize()
    final = bsp.pinn_residual_fwd_bwd(bsp.PinnNet(params.data, *spec), p, Xf[:8192].contiguous(),
                                      Xe[:512].contiguous(), Xb[:256].contiguous())[0]
    info = {"steps": step, "epochs": epoch, "seconds": time.time() - t0,
            "final_loss3": [float(v) for v in final.cpu()], "history": hist}
    return bsp.PinnNet(params.data.clone(), *spec), info


def train_call_network(cfg: dict, epochs_hi: int = 5000, epochs_lo: int = 800,
                       precision_train: int = bsp.PREC_FP32, precision_eval: int = bsp.PREC_BF16):
    """The network coarse of the 1024-node call workload: trained on that call
    (FP32 training), evaluated with `precision_eval`."""
    p = option_params(cfg)
    net, info = train(p, cfg["n_in"], cfg["depth"], cfg["width"], precision_train,
                      epochs_hi=epochs_hi, epochs_lo=epochs_lo)
    net.precision = precision_eval
    return net, {k: v for k, v in info.items() if k != "history"}


def train_on_data(p: dict, X, y, n_in: int, depth: int, width: int,
                  precision: int = bsp.PREC_FP32, batch: int = 8192, epochs_hi: int = 5000,
                  epochs_lo: int = 800, lr_hi: float = 1e-2, lr_lo: float = 1e-3,
                  seed: int = SEED, init_seed: int = 0):
    """A network fitted to data alone (no PDE terms): the same MLP and Adam
    schedule as train(), with the loss the mean squared error between the
    network and the targets y at the points X (float32 [n, n_in], v = V/K
    targets [n]).  The gradient comes from the residual kernel with only its
    value-matching set (n_f = n_b = 0).  Returns (PinnNet, info dict)."""
    dev = torch.device("cuda")
    X = torch.as_tensor(X, dtype=torch.float32, device=dev).contiguous()
    y = torch.as_tensor(y, dtype=torch.float32, device=dev).contiguous()
    n = X.shape[0]
    if y.numel() != n or X.shape[1] != n_in:
        raise ValueError("X must be [n, n_in] and y [n]")
    batch = min(batch, n)
    params = torch.nn.Parameter(torch.tensor(xavier_normal(n_in, depth, width, init_seed),
                                             device=dev))
    spec = (n_in, depth, width, precision)
    net = bsp.PinnNet(params.data, *spec)
    ws = torch.empty(bsp.pinn_residual_workspace_size(net, 0, batch, 0), dtype=torch.uint8,
                     device=dev)
    empty = torch.empty((0, n_in), dtype=torch.float32, device=dev)
    opt = torch.optim.Adam([params], lr=lr_hi)
    per_epoch = n // batch
    t0 = time.time()
    step = 0
    for epoch in range(epochs_hi + epochs_lo):
        if epoch == epochs_hi:
            for gopt in opt.param_groups:
                gopt["lr"] = lr_lo
        for idx in minibatch_indices(n, batch, epoch, seed):
            i = torch.as_tensor(idx, device=dev)
            opt.zero_grad(set_to_none=True)
            loss = DataLoss.apply(params, spec, p, X[i].contiguous(), y[i].contiguous(), empty,
                                  ws)
            loss.backward()
            opt.step()
            step += 1
    torch.cuda.synchronize()
    m = min(n, batch)
    final = bsp.pinn_residual_fwd_bwd(bsp.PinnNet(params.data, *spec), p, empty, X[:m].contiguous(),
                                      empty, y_e=y[:m].contiguous())[0]
    info = {"steps": step, "epochs": epochs_hi + epochs_lo, "per_epoch": per_epoch,
            "seconds": time.time() - t0, "final_data_mse": float(final[1])}
    return bsp.PinnNet(params.data.clone(), *spec), info
