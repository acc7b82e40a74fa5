"""Helpers shared by the GPU tests (parity metrics, device setup)."""
import numpy as np
import torch


def cuda():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch.device("cuda")


def normwise(got, ref):
    """max |got - ref| / max |ref| (relative to the solution's scale)."""
    got, ref = np.asarray(got), np.asarray(ref)
    scale = max(np.max(np.abs(ref)), 1e-300)
    return float(np.max(np.abs(got - ref)) / scale)


def to_dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def say(*args):
    print(*args, flush=True)


def network_grid(bsp, net, p, M, N):
    """The library's network values v(tau_n, S_j / K) on the Parareal grid,
    [N+1, M] float64 (pinn_forward on inputs built here)."""
    S = (np.arange(1, M + 1) * (p["s_max"] / (M + 1))) / p["K"]
    taus = np.arange(N + 1) * (p["T"] / N)
    T, X = np.meshgrid(taus, S, indexing="ij")
    X = torch.tensor(np.stack([T.ravel(), X.ravel()], 1), dtype=torch.float32, device="cuda")
    return bsp.pinn_forward(net, X).double().reshape(N + 1, M).cpu().numpy()
