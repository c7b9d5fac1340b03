"""pr_gram_noalloc (the Gram of Algorithm 1, step 1, without device
allocation) against pr_gram through the C ABI: bitwise the same G on two
calls in a row, the second smaller, in both precisions, plus the largest
shape its static scratch holds and its size limit."""
import numpy as np
import pytest

import workloads as W
from oracle import pod
from gpu_helpers import say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _cols(n, ncols, seed, f32):
    rng = np.random.Generator(np.random.PCG64(seed))
    Wm = rng.standard_normal((ncols, n ** 3))
    if f32:
        Wm = Wm.astype(np.float32).astype(np.float64)
    return Wm


def _check(ctx, n, ncols, seed, prec):
    import torch
    import paper_2601_10981_amd as pr
    say(f"no-alloc Gram n={n} ncols={ncols} precision={prec}")
    f32 = prec == W.PREC_MIXED
    prob = pr.problem_of(W.Problem(n=n, kappa=0.05, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0),
                                   precision=prec))
    Wm = _cols(n, ncols, seed, f32)
    Wd = to_dev(Wm, torch.float32 if f32 else torch.float64)
    used = ctx.scratch_bytes()
    G_na = torch.full((ncols, ncols), float("nan"), dtype=torch.float64, device="cuda")
    pr.pr_gram_noalloc(ctx, prob, Wd, G_na)
    torch.cuda.synchronize()
    assert ctx.scratch_bytes() == used      # no context scratch taken
    G_ref = pr.pr_gram(ctx, prob, Wd, ncols)
    torch.cuda.synchronize()
    a, b = to_np(G_na), to_np(G_ref)
    assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
    h = 2 * np.pi / n
    Go = pod.gram(Wm.T, h ** 3)
    rel = np.linalg.norm(a - Go) / np.linalg.norm(Go)
    say(f"  rel. Frobenius error vs the oracle Gram {rel:.2e}")
    assert rel <= (1e-6 if f32 else 1e-12)


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_10981_amd as pr
    c = pr.Context(0)
    yield c
    c.close()


def test_noalloc_gram_two_calls_second_smaller(ctx):
    _check(ctx, 40, 48, 11, W.PREC_F64)
    _check(ctx, 12, 5, 12, W.PREC_F64)


def test_noalloc_gram_mixed_two_calls(ctx):
    _check(ctx, 32, 33, 13, W.PREC_MIXED)
    _check(ctx, 8, 17, 14, W.PREC_MIXED)


def test_noalloc_gram_largest_partials(ctx):
    # 96^3 rows: 512 row chunks x 10 tile pairs, the scratch's full size
    _check(ctx, 96, 64, 15, W.PREC_F64)
    _check(ctx, 16, 3, 16, W.PREC_F64)


def test_noalloc_gram_rejects_too_many_columns(ctx):
    import torch
    import paper_2601_10981_amd as pr
    prob = pr.problem_of(W.Problem(n=8, kappa=0.05, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0)))
    Wd = torch.zeros(65 * 8 ** 3, dtype=torch.float64, device="cuda")
    G = torch.zeros((65, 65), dtype=torch.float64, device="cuda")
    with pytest.raises(pr.PrError) as e:
        pr.pr_gram_noalloc(ctx, prob, Wd, G)
    assert e.value.name == "PR_EINVAL"
