"""Helpers shared by the GPU tests (device tensors, oracle comparisons)."""
import numpy as np
import torch


def dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a, b):
    return abs(a - b) / max(1.0, abs(b))
