"""Shared helpers of the GPU tests (no method arithmetic here)."""
from __future__ import annotations

import numpy as np


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).reshape(-1).copy())
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def say(msg: str) -> None:
    print(msg, flush=True)
