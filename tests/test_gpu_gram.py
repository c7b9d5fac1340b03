"""GPU parity of the MFMA snapshot Gram (pr_gram, Algorithm 1 step 1)
against the plain product h^3 W^T W: FP64 to 1e-13 relative to the largest
entry, FP32 MFMA to 1e-5; integer-valued snapshots give the exact Gram."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_helpers import say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_10981_amd as pr
    c = pr.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,ncols", [(8, 1), (9, 16), (10, 17), (12, 33), (16, 48), (13, 64), (64, 16)])
def test_gram_f64(ctx, n, ncols):
    import torch
    import paper_2601_10981_amd as pr
    say(f"gram f64 n={n} ncols={ncols}")
    Wm = W.random_matrix(n ** 3, ncols, n + ncols)
    prob = pr.problem(n, 0.05, W.FLOW_ABC, (1, 1, 1))
    G = pr.pr_gram(ctx, prob, to_dev(Wm.T), ncols)
    torch.cuda.synchronize()
    h3 = (2 * math.pi / n) ** 3
    ref = h3 * (Wm.T @ Wm)
    Gn = to_np(G)
    assert np.max(np.abs(Gn - ref)) <= 1e-13 * np.max(np.abs(ref)), np.max(np.abs(Gn - ref))


@pytest.mark.parametrize("n,ncols", [(9, 16), (12, 40)])
def test_gram_f32_exact_on_integers(ctx, n, ncols):
    import torch
    import paper_2601_10981_amd as pr
    rng = np.random.Generator(np.random.PCG64(3))
    Wm = rng.integers(-3, 4, size=(n ** 3, ncols)).astype(np.float64)
    prob = pr.problem(n, 0.05, W.FLOW_ABC, (1, 1, 1), W.PREC_MIXED)
    G = pr.pr_gram(ctx, prob, to_dev(Wm.T, torch.float32), ncols)
    torch.cuda.synchronize()
    h3 = (2 * math.pi / n) ** 3
    # integer products and sums below 2^24 are exact in FP32; the scale by h^3 is one FP64 rounding
    assert np.max(np.abs(to_np(G) - h3 * (Wm.T @ Wm))) <= 1e-15 * h3 * np.max(np.abs(Wm.T @ Wm))


def test_gram_f32_random(ctx):
    import torch
    import paper_2601_10981_amd as pr
    n, ncols = 32, 16
    Wm = W.random_matrix(n ** 3, ncols, 4)
    prob = pr.problem(n, 0.05, W.FLOW_ABC, (1, 1, 1), W.PREC_MIXED)
    G = pr.pr_gram(ctx, prob, to_dev(Wm.T, torch.float32), ncols)
    torch.cuda.synchronize()
    W32 = Wm.astype(np.float32).astype(np.float64)
    h3 = (2 * math.pi / n) ** 3
    ref = h3 * (W32.T @ W32)
    assert np.max(np.abs(to_np(G) - ref)) <= 1e-5 * np.max(np.abs(ref))
