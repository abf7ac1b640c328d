"""Helpers shared by the GPU tests: device check, oracle<->device field layout."""
import numpy as np
import pytest

from oracle import tensors


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1712_05145_amd import ffth
    ffth.load()   # raises when libffth.so is not built
    return torch


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def voigt6(t):
    """(3,3,...) oracle field -> (6,...) tensor components."""
    return tensors.voigt6_from_field(t)


def full(f6):
    return tensors.field_from_voigt6(f6)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    w = np.ones(a.shape[0]) if a.shape[0] != 6 else np.array([1, 1, 1, 2, 2, 2], float)
    shp = (-1,) + (1,) * (a.ndim - 1)
    num = np.sqrt(np.sum(w.reshape(shp) * (a - b) ** 2))
    den = np.sqrt(np.sum(w.reshape(shp) * b ** 2))
    return num / den if den > 0 else num
