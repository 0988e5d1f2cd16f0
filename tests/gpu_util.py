"""Helpers for the GPU parity tests (imported only by tests marked gpu)."""
import numpy as np
import torch


def dev():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch.device("cuda:0")


def f32(a):
    """Round host data to FP32 once; both sides then see identical values."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def to_gpu(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def say(*args):
    print(*args, flush=True)
