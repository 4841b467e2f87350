"""Helpers for the GPU parity tests: device checks and oracle/GPU conversions."""
import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2210_00947_amd import mgar as M
    M.lib()  # raises if the HIP library is missing: no fallback
    return torch


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a, b):
    """max-abs error relative to the max-abs of the reference."""
    a, b = np.asarray(a), np.asarray(b)
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / (s if s > 0 else 1.0))


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    s = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (s if s > 0 else 1.0))


def masked_random(n, fixed, seed):
    import workloads as W
    v = W.random_vector(n, seed)
    v[fixed] = 0.0
    return v
