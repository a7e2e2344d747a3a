"""Helpers shared by the GPU tests: layout conversion and error measures."""
import sys

import numpy as np
import torch


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def to_dev(a):
    """(N, 3) numpy -> (3, N) float64 CUDA tensor; (N,) -> (N,)."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 2:
        a = a.T
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def to_host(t):
    """(3, N) tensor -> (N, 3) numpy."""
    a = t.detach().cpu().numpy()
    return a.T.copy() if a.ndim == 2 else a


def rel_rows(got, ref):
    """Per-row |got - ref| / |ref| for (N, 3) arrays."""
    return np.sqrt(((got - ref) ** 2).sum(1)) / np.sqrt((ref ** 2).sum(1))


def rel_norm(got, ref):
    return float(np.sqrt(np.sum((got - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))
