"""Helpers shared by the GPU tests: device tensors and tolerances."""

import numpy as np
import torch

# normwise tolerances on values (the integer RNG pieces are compared exactly)
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def dev(x, dtype=None):
    """Column-major device copy of a numpy array."""
    t = torch.from_numpy(np.asarray(x))
    if dtype is not None:
        t = t.to(dtype)
    if t.dim() == 2:
        t = t.t().contiguous().t()
    return t.cuda()


def host(t):
    return t.detach().cpu().double().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def bits_of(t):
    """Exact float64 view of a device tensor's values (fp32 promoted exactly)."""
    return t.detach().cpu().double().numpy()
