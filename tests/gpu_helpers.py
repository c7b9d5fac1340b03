"""Shared helpers of the GPU tests (no method arithmetic here: the round-off
envelope only re-runs the oracle on perturbed inputs)."""
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


def roundoff_envelope(prob, opts, u0, base, kmax, seeds=(0, 1)):
    """How far the oracle's own iterates move when every snapshot matrix is
    perturbed by one unit in the last place (relative 2.2e-16, seeded): the
    POD modes near the rank cut (lambda ~ 1e-13 lambda_1) are fixed by the
    data only to about eps lambda_1 / gap, so intermediate iterates of any
    FP64 implementation agree only to this envelope. Returns env[k]."""
    from oracle import parareal, pod
    orig = pod.gram
    env = [0.0] * (kmax + 1)
    try:
        for sd in seeds:
            rng = np.random.Generator(np.random.PCG64(1000 + sd))

            def g(Wm, h3):
                return orig(Wm * (1.0 + 2.2e-16 * rng.uniform(-1.0, 1.0, Wm.shape)), h3)
            pod.gram = g
            alt = parareal.solve(prob, opts, u0, keep_history=True)
            pod.gram = orig
            for k in range(1, kmax + 1):
                e = max(rel_l2(a, b) for a, b in zip(alt.history[k], base.history[k]))
                env[k] = max(env[k], e)
    finally:
        pod.gram = orig
    return env
