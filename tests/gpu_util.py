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


ELEMENT_FACTOR = 10.0


def close(got, ref, tol, factor=ELEMENT_FACTOR):
    """Relative 2-norm error within tol AND every element within factor * tol of the largest
    reference magnitude (so that a few bad elements cannot hide inside the norm)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = float(np.abs(ref).max()) if ref.size else 0.0
    emax = float(np.abs(got - ref).max()) if ref.size else 0.0
    return rel2(got, ref) <= tol and emax <= factor * tol * scale


def max_element(got, ref):
    """Largest element error relative to the largest reference magnitude."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(got - ref).max() / np.abs(ref).max())
