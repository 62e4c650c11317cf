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


def delta_ok(orc, E, beta, d_gpu, d_ref, rho=0.5):
    """The GPU increment equals the reference's halving result, or (where the FP64 rounding
    of the weight sums decides the last halvings) is itself a root of ESS = rho P to FP64
    precision."""
    width = (1.0 - beta) * 2.0 ** -50
    if abs(d_gpu - d_ref) <= 4 * width + 1e-12 * d_ref:
        return True
    target = rho * len(E)
    return abs(orc.ess(E, d_gpu)[0] / target - 1.0) <= 1e-12
