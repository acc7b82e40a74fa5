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
