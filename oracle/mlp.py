"""FP64 oracle for the physics-informed network (paper Sec. 3.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network: ``n_in`` inputs -> ``depth`` hidden layers of ``width`` units with
tanh -> one linear output.  Inputs are ``(tau, x)`` with time to maturity
``tau`` and ``x = S/K``, or ``(tau, x, sigma, r)`` for a network
parametrised by the model coefficients.  The output is ``v = V/K``.

Parameters are one flat vector in the order of ``torch.nn.Linear`` layers:
``W1[w][n_in], b1[w], W2[w][w], b2[w], ..., Wd[w][w], bd[w], Wo[1][w], bo[1]``.

Readings of the paper used here:
  * The paper's network uses ReLU (Sec. 3.3); its second derivative vanishes
    almost everywhere, which would drop the diffusion term from the residual
    computed by automatic differentiation.  The hidden activation is tanh.
  * Eq. (1) is written in calendar time t; in tau = T - t and in the
    dimensionless variables v = V/K, x = S/K it becomes the residual
        f = v_tau - sigma^2 x^2 v_xx / 2 - r x v_x + r v,
    which does not depend on K.
  * Eqs. (11)-(14): the loss is the unweighted sum of three mean squares:
    the residual at interior points, the expiry condition (tau = 0) at
    terminal points, the Dirichlet values at boundary points.  Eq. labels in
    the prose of Sec. 3.3 swap the terminal and boundary conditions; the
    terminal points use eq. (2) and the boundary points eqs. (3)-(4).
  * The derivatives the paper takes by automatic differentiation are here
    forward-mode streams (value, d/dtau, d/dx, d2/dx2) carried through every
    layer, and the gradient of the loss is a hand-written reverse pass
    through those streams.

Pins (tests/test_oracle_mlp.py): torch float64 ``nn.Sequential`` forward and
``autograd.grad`` derivatives; the loss gradient against torch autograd and
against central finite differences.

The bfloat16 option of loss_grad (operand_round=bf16_round) rounds both
operands of every hidden-layer product, as the matrix-core pass does, and
computes everything else in float64.  Pins: bf16_round against torch's
bfloat16 conversion (ties included); no change for a network without hidden
products; the value-set losses against a torch float64 forward with
torch-rounded operands.  Where the backward products take rounded operands
has no independent pin (parity unpinned for that placement beyond the
agreement with the device pass).
"""
from __future__ import annotations

import numpy as np


def n_params(n_in: int, depth: int, width: int) -> int:
    return width * n_in + width + (depth - 1) * (width * width + width) + width + 1


def unpack(theta, n_in, depth, width):
    """Split the flat parameter vector into [(W, b), ...] (output layer last)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == n_params(n_in, depth, width), (theta.size, n_in, depth, width)
    layers, o = [], 0
    fan_in = n_in
    for _ in range(depth):
        W = theta[o:o + width * fan_in].reshape(width, fan_in)
        o += width * fan_in
        b = theta[o:o + width]
        o += width
        layers.append((W, b))
        fan_in = width
    W = theta[o:o + width].reshape(1, width)
    o += width
    b = theta[o:o + 1]
    layers.append((W, b))
    return layers


def forward(theta, X, n_in, depth, width):
    """Network value v at the points X [n, n_in]."""
    X = np.asarray(X, dtype=np.float64)
    layers = unpack(theta, n_in, depth, width)
    a = X
    for W, b in layers[:-1]:
        a = np.tanh(a @ W.T + b)
    Wo, bo = layers[-1]
    return (a @ Wo.T + bo)[:, 0]


def bf16_round(x):
    """x rounded to bfloat16 (8 significant bits, to nearest, ties to even)
    through float32, as a float32 value converts to bfloat16."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _identity(x):
    return x


def _hidden_streams(layers, X, rnd=_identity):
    """Forward-mode streams through the hidden layers.

    Returns per layer the cache (a, z_t, z_x, z_xx) and the final
    (a, a_t, a_x, a_xx).  For a = tanh(z), s = 1 - a^2:
        a_t = s z_t,  a_x = s z_x,  a_xx = s z_xx - 2 a s z_x^2.
    rnd is applied to both operands of every hidden-layer product (the
    identity, or bf16_round for operands rounded to bfloat16).
    """
    n = X.shape[0]
    W1, b1 = layers[0]
    z = X @ W1.T + b1
    z_t = np.broadcast_to(W1[:, 0], z.shape).copy()
    z_x = np.broadcast_to(W1[:, 1], z.shape).copy()
    z_xx = np.zeros_like(z)
    caches = []
    for li in range(len(layers) - 1):
        if li > 0:
            W, b = layers[li]
            Wr = rnd(W)
            z = rnd(a) @ Wr.T + b
            z_t = rnd(a_t) @ Wr.T
            z_x = rnd(a_x) @ Wr.T
            z_xx = rnd(a_xx) @ Wr.T
        a = np.tanh(z)
        s = 1.0 - a * a
        caches.append((a, z_t, z_x, z_xx))
        a_t = s * z_t
        a_x = s * z_x
        a_xx = s * z_xx - 2.0 * a * s * z_x * z_x
    assert a.shape[0] == n
    return caches, (a, a_t, a_x, a_xx)


def streams(theta, X, n_in, depth, width):
    """v, v_tau, v_x, v_xx at the points X."""
    X = np.asarray(X, dtype=np.float64)
    layers = unpack(theta, n_in, depth, width)
    _, (a, a_t, a_x, a_xx) = _hidden_streams(layers, X)
    Wo, bo = layers[-1]
    wo = Wo[0]
    return a @ wo + bo[0], a_t @ wo, a_x @ wo, a_xx @ wo


def _coeffs(X, sigma, r):
    """sigma and r per point: given scalars, or columns 2 and 3 of X."""
    if sigma is None:
        return X[:, 2], X[:, 3]
    n = X.shape[0]
    return np.full(n, float(sigma)), np.full(n, float(r))


def residual_from_streams(v, v_t, v_x, v_xx, x, sigma, r):
    """f = v_tau - sigma^2 x^2 v_xx / 2 - r x v_x + r v: eq. (1) in tau = T - t,
    v = V/K, x = S/K."""
    return v_t - 0.5 * sigma * sigma * x * x * v_xx - r * x * v_x + r * v


def residual(theta, X, n_in, depth, width, sigma=None, r=None):
    """PDE residual of the network at the points X (sigma, r given, or taken
    from X[:, 2], X[:, 3] for a parametrised network)."""
    X = np.asarray(X, dtype=np.float64)
    v, v_t, v_x, v_xx = streams(theta, X, n_in, depth, width)
    sg, rr = _coeffs(X, sigma, r)
    return residual_from_streams(v, v_t, v_x, v_xx, X[:, 1], sg, rr)


def terminal_target(X, is_put):
    """Eq. (2) in v = V/K, x = S/K at tau = 0: max(x-1, 0) (call), max(1-x, 0) (put)."""
    x = np.asarray(X, dtype=np.float64)[:, 1]
    return np.maximum(1.0 - x, 0.0) if is_put else np.maximum(x - 1.0, 0.0)


def boundary_target(X, is_put, r=None):
    """Eqs. (3)-(4) in v units.  A point with x == 0 is on the lower boundary
    (call 0, put exp(-r tau)); any other boundary point is on the upper one
    (call x - exp(-r tau), put 0)."""
    X = np.asarray(X, dtype=np.float64)
    tau, x = X[:, 0], X[:, 1]
    rr = X[:, 3] if r is None else np.full(X.shape[0], float(r))
    disc = np.exp(-rr * tau)
    lower = x == 0.0
    if is_put:
        return np.where(lower, disc, 0.0)
    return np.where(lower, 0.0, x - disc)


def _mean(a):
    """Mean of the squared terms; an empty set of points contributes 0."""
    return float(np.mean(a)) if a.size else 0.0


def _targets(X_e, X_b, is_put, r, y_e, y_b):
    """Value targets of the terminal and boundary sets: given, or eqs. (2)-(4)."""
    ye = terminal_target(X_e, is_put) if y_e is None else np.asarray(y_e, dtype=np.float64)
    yb = boundary_target(X_b, is_put, r) if y_b is None else np.asarray(y_b, dtype=np.float64)
    return ye, yb


def loss3(theta, X_f, X_e, X_b, n_in, depth, width, is_put=False, sigma=None, r=None,
          y_e=None, y_b=None):
    """(MSE_f, MSE_exp, MSE_b), eqs. (12)-(14); their sum is eq. (11).  y_e, y_b:
    value targets replacing eq. (2) at the X_e points and eqs. (3)-(4) at the
    X_b points (a network fitted to data: n_f = 0 and y_e the data)."""
    f = residual(theta, X_f, n_in, depth, width, sigma, r)
    ve = forward(theta, X_e, n_in, depth, width)
    vb = forward(theta, X_b, n_in, depth, width)
    ye, yb = _targets(X_e, X_b, is_put, r, y_e, y_b)
    return (_mean(f * f), _mean((ve - ye) ** 2), _mean((vb - yb) ** 2))


def loss_grad(theta, X_f, X_e, X_b, n_in, depth, width, is_put=False, sigma=None, r=None,
              y_e=None, y_b=None, operand_round=None, with_loss=False):
    """Gradient of MSE_f + MSE_exp + MSE_b with respect to the flat parameters
    (targets y_e, y_b as in loss3).

    operand_round (e.g. bf16_round) is applied to both operands of every
    hidden-layer product, forward (W a_s) and backward (W^T zbar_s and
    zbar_s a_prev_s^T), and nowhere else: the arithmetic of a pass whose
    hidden-layer products take bfloat16 operands.  with_loss: return
    ((MSE_f, MSE_exp, MSE_b), gradient), the losses from the same streams.

    Reverse pass, written by hand, through the value and derivative streams.
    Output adjoints per point (gv, gt, gx, gxx) for (v, v_tau, v_x, v_xx):
      interior:  with df = 2 f / n_f:  gv = r df, gt = df, gx = -r x df,
                 gxx = -sigma^2 x^2 df / 2;
      terminal / boundary: gv = 2 (v - y) / n, the others zero.
    Through a = tanh(z), s = 1 - a^2, given adjoints (A, At, Ax, Axx) of
    (a, a_t, a_x, a_xx):
      zbar_t  = s At
      zbar_x  = s Ax - 4 a s z_x Axx
      zbar_xx = s Axx
      zbar    = s [A - 2 a (z_t At + z_x Ax + z_xx Axx) - 2 z_x^2 (1 - 3 a^2) Axx]
    Through z = W a_prev + b (and z_* = W a_prev_*):
      dW += zbar a_prev^T + zbar_t a_prev_t^T + zbar_x a_prev_x^T + zbar_xx a_prev_xx^T,
      db += sum zbar, and the adjoints of a_prev_* are W^T zbar_*.
    In the first layer z_t = W[:, 0] and z_x = W[:, 1], so
      dW[:, 0] += sum zbar_t and dW[:, 1] += sum zbar_x.
    """
    X_f, X_e, X_b = (np.asarray(a, dtype=np.float64) for a in (X_f, X_e, X_b))
    layers = unpack(theta, n_in, depth, width)
    n_f, n_e, n_b = X_f.shape[0], X_e.shape[0], X_b.shape[0]
    X = np.concatenate([X_f, X_e, X_b], axis=0)
    rnd = _identity if operand_round is None else operand_round
    caches, (a, a_t, a_x, a_xx) = _hidden_streams(layers, X, rnd)
    Wo, bo = layers[-1]
    wo = Wo[0]
    v = a @ wo + bo[0]
    v_t, v_x, v_xx = a_t @ wo, a_x @ wo, a_xx @ wo

    n = X.shape[0]
    losses = [0.0, 0.0, 0.0]
    ye, yb = _targets(X_e, X_b, is_put, r, y_e, y_b)
    gv, gt, gx, gxx = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    if n_f:
        sl = slice(0, n_f)
        sg, rr = _coeffs(X_f, sigma, r)
        x = X_f[:, 1]
        f = residual_from_streams(v[sl], v_t[sl], v_x[sl], v_xx[sl], x, sg, rr)
        losses[0] = _mean(f * f)
        df = 2.0 * f / n_f
        gv[sl] = rr * df
        gt[sl] = df
        gx[sl] = -rr * x * df
        gxx[sl] = -0.5 * sg * sg * x * x * df
    if n_e:
        sl = slice(n_f, n_f + n_e)
        losses[1] = _mean((v[sl] - ye) ** 2)
        gv[sl] = 2.0 * (v[sl] - ye) / n_e
    if n_b:
        sl = slice(n_f + n_e, n)
        losses[2] = _mean((v[sl] - yb) ** 2)
        gv[sl] = 2.0 * (v[sl] - yb) / n_b

    grads = []
    g_wo = gv @ a + gt @ a_t + gx @ a_x + gxx @ a_xx
    g_bo = np.array([gv.sum()])
    A, At, Ax, Axx = np.outer(gv, wo), np.outer(gt, wo), np.outer(gx, wo), np.outer(gxx, wo)
    for li in range(len(layers) - 2, -1, -1):
        a_c, z_t, z_x, z_xx = caches[li]
        s = 1.0 - a_c * a_c
        zb_t = s * At
        zb_x = s * Ax - 4.0 * a_c * s * z_x * Axx
        zb_xx = s * Axx
        zb = s * (A - 2.0 * a_c * (z_t * At + z_x * Ax + z_xx * Axx)
                  - 2.0 * z_x * z_x * (1.0 - 3.0 * a_c * a_c) * Axx)
        W, _ = layers[li]
        if li > 0:
            p_a, p_zt, p_zx, p_zxx = caches[li - 1]
            p_s = 1.0 - p_a * p_a
            pa_t, pa_x = p_s * p_zt, p_s * p_zx
            pa_xx = p_s * p_zxx - 2.0 * p_a * p_s * p_zx * p_zx
            gW = (rnd(zb).T @ rnd(p_a) + rnd(zb_t).T @ rnd(pa_t) + rnd(zb_x).T @ rnd(pa_x)
                  + rnd(zb_xx).T @ rnd(pa_xx))
            Wr = rnd(W)
            A, At, Ax, Axx = rnd(zb) @ Wr, rnd(zb_t) @ Wr, rnd(zb_x) @ Wr, rnd(zb_xx) @ Wr
        else:
            gW = zb.T @ X
            gW[:, 0] += zb_t.sum(axis=0)
            gW[:, 1] += zb_x.sum(axis=0)
        grads.append((gW, zb.sum(axis=0)))
    grads.reverse()
    flat = [np.concatenate([gW.ravel(), gb]) for gW, gb in grads]
    flat.append(np.concatenate([g_wo, g_bo]))
    grad = np.concatenate(flat)
    return (tuple(losses), grad) if with_loss else grad


def grid_values(theta, n_in, depth, width, K, taus, S, sigma=None, r=None):
    """Network prediction in price units, K * v(tau_n, S_j / K), shape [len(taus), len(S)].

    This is the coarse propagator's view of the network (Sec. 3.3: the network
    returns the option price at the end of a time slice)."""
    taus = np.asarray(taus, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    T, Sg = np.meshgrid(taus, S / K, indexing="ij")
    cols = [T.ravel(), Sg.ravel()]
    if n_in == 4:
        cols += [np.full(T.size, float(sigma)), np.full(T.size, float(r))]
    X = np.stack(cols, axis=1)
    return K * forward(theta, X, n_in, depth, width).reshape(T.shape)
