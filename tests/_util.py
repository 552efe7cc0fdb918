"""Shared helpers of the test-suite (no method arithmetic)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    elif t.is_complex():
        t = t.to(torch.complex64)
    else:
        t = t.to(torch.float32)
    return t.cuda()


def to_host(t):
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)
