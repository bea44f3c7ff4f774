"""Helpers for the GPU parity tests (they call the HIP library through its C ABI)."""
import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run them with -m gpu on an MI355X)")


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel2(a, b):
    """Relative 2-norm error |a - b| / |b|."""
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def awkward_config(n=40, seed=5):
    """Spheres with overlaps, heights below a, on and below the wall, coincident clamped pairs."""
    rng = np.random.default_rng(seed)
    pos = np.column_stack([rng.uniform(0, 7, n), rng.uniform(0, 7, n), rng.uniform(0.2, 3.0, n)])
    pos[1, 2] = 0.0
    pos[2, 2] = -0.4
    pos[3, :2] = pos[4, :2]
    pos[3, 2], pos[4, 2] = 0.5, 0.8     # identical after clamping to z = a
    pos[5] = pos[6] + np.array([0.3, 0.0, 0.0])
    return pos
