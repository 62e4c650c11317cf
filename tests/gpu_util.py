"""Helpers shared by the GPU parity tests (device buffers through PyTorch)."""
import sys

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def say(*a):
    """Name the case before a GPU step (the output survives a lost box)."""
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def energy_constant(spec) -> float:
    """Theta-independent part of the negative log-likelihood (numpy/scipy, test side)."""
    from scipy.special import gammaln
    y = np.asarray(spec.y, dtype=np.float64)
    if spec.noise_kind == "gauss":
        return 0.5 * len(y) * np.log(2 * np.pi * spec.sigma ** 2)
    ylny = np.where(y > 0, y * np.log(np.where(y > 0, y, 1.0)), 0.0)
    return float(np.sum(y - ylny + gammaln(y + 1.0)))


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)
