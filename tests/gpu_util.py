"""Helpers for the GPU parity tests: numpy <-> device tensors, error norms."""

import sys

import numpy as np


def dev():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.fail("GPU test run without a visible GPU")
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
