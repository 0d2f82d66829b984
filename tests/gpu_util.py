"""Helpers for the GPU tests (the `gpu` marker; skipped without a device)."""
import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(a):
    import torch
    a = np.asarray(a)
    if np.iscomplexobj(a):
        b = np.empty(a.shape[:-1] + (2 * a.shape[-1],))
        b[..., 0::2] = a.real
        b[..., 1::2] = a.imag
        a = b
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def from_dev(t, complex_=False):
    a = t.detach().cpu().numpy()
    if complex_:
        return a[..., 0::2] + 1j * a[..., 1::2]
    return a


def quad_scale(parts):
    a, b = parts
    return np.abs(a) + np.abs(b)
