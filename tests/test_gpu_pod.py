"""GPU parity of POD_Mode (pr_pod_build, Algorithm 1) against the oracle.

Gram eigenvalues (which pin the MFMA Gram), ranks, projectors R R^T M and
M-orthonormality. Ranks are integers decided in FP64 on both sides and must
match exactly; bases are compared through projectors (eigenvector signs and
rotations inside degenerate eigenspaces are not unique) and column by column
for well-separated modes.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fd, pod
from gpu_helpers import rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_10981_amd as pr
    c = pr.Context(0)
    yield c
    c.close()


def _snapshots(n, ncols, seed, decay=1.0):
    """Snapshots of a real fine trajectory (smooth, decaying spectrum)."""
    op = fd.Operator(n, 0.05, W.FLOW_ABC, (1.0, 1.0, 1.0))
    u0 = W.fourier_field(n, seed, n_modes=8, kmax=3.0) + 0.01 * W.random_field(n, seed + 100)
    _, Wm = fd.fine_propagate(op, u0, 0.01, (ncols - 1) * 2, 2)
    return Wm


def _random_block(n, ncols, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return W.random_matrix(n ** 3, ncols, seed) * np.logspace(0, -4, ncols)[None, :]


def _gpu_pod(ctx, n, blocks, gamma, cap, prec=W.PREC_F64, valid=None, force_m=-1):
    import torch
    import paper_2601_10981_amd as pr
    fdt = torch.float32 if prec == W.PREC_MIXED else torch.float64
    prob = pr.problem(n, 0.05, W.FLOW_ABC, (1, 1, 1), prec)
    dblocks = [to_dev(b.T, fdt) for b in blocks]   # (cols, N_g)
    R = torch.empty((cap, n ** 3), dtype=fdt, device="cuda")
    m = torch.zeros(1, dtype=torch.int32, device="cuda")
    ncols = sum(b.shape[1] for b in blocks)
    lam = torch.empty(ncols, dtype=torch.float64, device="cuda")
    dvalid = None
    if valid is not None:
        dvalid = [None if v is None else torch.tensor([v], dtype=torch.int32, device="cuda")
                  for v in valid]
    pr.pr_pod_build(ctx, [dict(prob=prob, blocks=dblocks, gamma=gamma, cap=cap, R_out=R,
                               m_out=m, lambda_out=lam, block_valid=dvalid, force_m=force_m)])
    torch.cuda.synchronize()
    return to_np(R).reshape(cap, -1).T, int(m.item()), to_np(lam)


def _proj(R, h3):
    return h3 * (R @ R.T)


@pytest.mark.parametrize("n,ncols,gamma,cap", [(12, 16, 1 - 5e-6, 10), (10, 33, 0.9999, 12),
                                                (8, 64, 1.0, 31), (20, 7, 1 - 5e-6, 5)])
def test_pod_parity_f64(ctx, n, ncols, gamma, cap):
    say(f"pod parity n={n} cols={ncols}")
    Wm = _snapshots(n, ncols, seed=n)
    h3 = (2 * math.pi / n) ** 3
    Ro, mo, lo = pod.pod_mode(Wm, gamma, h3, cap)
    Rg, mg, lg = _gpu_pod(ctx, n, [Wm], gamma, cap)
    assert mg == mo
    assert np.max(np.abs(lg - lo)) <= 1e-12 * lo[0]
    P_o = _proj(Ro, h3)
    P_g = _proj(Rg[:, :mg], h3)
    # columns beyond m are zero
    assert np.all(Rg[:, mg:] == 0)
    assert np.max(np.abs(h3 * (Rg[:, :mg].T @ Rg[:, :mg]) - np.eye(mg))) <= 1e-13
    # projector agreement is limited by the conditioning of the trailing mode
    gap = lo[mg - 1] - (lo[mg] if mg < len(lo) else 0.0)
    tol = max(1e-12, 50 * 2.2e-16 * lo[0] / max(gap, 1e-300))
    assert np.max(np.abs(P_g - P_o)) <= tol
    # well-separated leading modes agree column by column (sign convention)
    for j in range(min(mg, 3)):
        assert rel_l2(Rg[:, j], Ro[:, j]) <= 1e-10


def test_pod_random_block_projector(ctx):
    n, ncols = 9, 20
    Wm = _random_block(n, ncols, 5)
    h3 = (2 * math.pi / n) ** 3
    Ro, mo, lo = pod.pod_mode(Wm, 1.0, h3, 20)
    Rg, mg, lg = _gpu_pod(ctx, n, [Wm], 1.0, 20)
    assert mg == mo == 20
    assert np.max(np.abs(lg - lo)) <= 1e-12 * lo[0]
    assert np.max(np.abs(_proj(Rg[:, :mg], h3) - _proj(Ro, h3))) <= 1e-11


def test_pod_constructed_spectrum(ctx):
    n = 8
    h3 = (2 * math.pi / n) ** 3
    D = np.array([10.0, 3.0, 1.0, 0.3, 0.1, 0.01, 1e-4, 1e-9])
    Q, _ = np.linalg.qr(W.random_matrix(n ** 3, len(D), 1))
    Q = Q / math.sqrt(h3)
    V, _ = np.linalg.qr(W.random_matrix(len(D), len(D), 2))
    Wm = Q @ np.diag(D) @ V.T
    _, m, lam = _gpu_pod(ctx, n, [Wm], 0.99, 10)
    assert m == 4
    assert np.max(np.abs(lam - D ** 2)) <= 1e-12 * D[0] ** 2
    _, m, _ = _gpu_pod(ctx, n, [Wm], 0.99, 3)
    assert m == 3
    _, m, _ = _gpu_pod(ctx, n, [Wm], 1.0, 10)
    assert m == 7
    _, m, _ = _gpu_pod(ctx, n, [Wm], 1.0, 10, force_m=2)
    assert m == 2


def test_pod_blocks_with_device_valid_counts(ctx):
    n = 10
    h3 = (2 * math.pi / n) ** 3
    B = [_snapshots(n, 6, s) for s in (3, 4, 5)]
    valid = [4, None, 2]
    Wcat = np.concatenate([B[0][:, :4], B[1], B[2][:, :2]], axis=1)
    Ro, mo, lo = pod.pod_mode(Wcat, 1 - 1e-10, h3, 8)
    Rg, mg, lg = _gpu_pod(ctx, n, B, 1 - 1e-10, 8, valid=valid)
    assert mg == mo
    nz = np.sort(lg)[::-1][:Wcat.shape[1]]
    assert np.max(np.abs(nz - lo)) <= 1e-12 * lo[0]
    gap = lo[mg - 1] - lo[mg]
    assert np.max(np.abs(_proj(Rg[:, :mg], h3) - _proj(Ro, h3))) <= max(1e-12, 100 * 2.2e-16 * lo[0] / gap)


def test_pod_zero_input(ctx):
    R, m, lam = _gpu_pod(ctx, 8, [np.zeros((512, 5))], 0.99, 4)
    assert m == 0 and np.all(R == 0)


def test_pod_batch_equals_single(ctx):
    import torch
    import paper_2601_10981_amd as pr
    n = 12
    prob = pr.problem(n, 0.05, W.FLOW_ABC, (1, 1, 1))
    sets = [_snapshots(n, 16, s) for s in (7, 8, 9)]
    Rs = [torch.empty((10, n ** 3), dtype=torch.float64, device="cuda") for _ in sets]
    ms = [torch.zeros(1, dtype=torch.int32, device="cuda") for _ in sets]
    pr.pr_pod_build(ctx, [dict(prob=prob, blocks=[to_dev(Wm.T)], gamma=1 - 5e-6, cap=10,
                               R_out=R, m_out=m) for Wm, R, m in zip(sets, Rs, ms)])
    torch.cuda.synchronize()
    for Wm, R, m in zip(sets, Rs, ms):
        Rg, mg, _ = _gpu_pod(ctx, n, [Wm], 1 - 5e-6, 10)
        assert mg == int(m.item())
        assert np.array_equal(Rg, to_np(R).reshape(10, -1).T)


def test_pod_mixed_precision_leading_modes(ctx):
    n = 16
    Wm = _snapshots(n, 16, 11)
    h3 = (2 * math.pi / n) ** 3
    Ro, mo, lo = pod.pod_mode(Wm, 1 - 5e-6, h3, 10, tau_r=pod.TAU_R_F32)
    Rg, mg, lg = _gpu_pod(ctx, n, [Wm], 1 - 5e-6, 10, prec=W.PREC_MIXED)
    assert abs(mg - mo) <= 1
    # Gram entries of the FP32 path within 1e-5 lambda_1
    k = min(mg, mo)
    assert np.max(np.abs(lg[:3] - lo[:3])) <= 1e-5 * lo[0]
    # leading well-separated modes: projectors within 1e-5
    lead = [j for j in range(k - 1) if lo[j] - lo[j + 1] > 1e-2 * lo[0]]
    if lead:
        L_ = lead[-1] + 1
        assert np.max(np.abs(_proj(Rg[:, :L_], h3) - _proj(Ro[:, :L_], h3))) <= 1e-5
    assert np.max(np.abs(h3 * (Rg[:, :mg].T @ Rg[:, :mg]) - np.eye(mg))) <= 1e-5


@pytest.mark.parametrize("prec", [W.PREC_F64, W.PREC_MIXED], ids=["f64", "mixed"])
def test_pod_masked_columns_are_never_read(ctx, prec):
    """Columns beyond a block's device valid count hold NaN: the Gram, the
    eigenproblem and the mode formation skip them, so the result is bitwise
    that of the same blocks with those columns zeroed."""
    n = 10
    B = [_snapshots(n, 6, s) for s in (3, 4, 5)]
    valid = [4, None, 2]
    Bz = [b.copy() for b in B]
    Bn = [b.copy() for b in B]
    for b_z, b_n, v in zip(Bz, Bn, valid):
        if v is not None:
            b_z[:, v:] = 0.0
            b_n[:, v:] = np.nan
    Rz, mz, lz = _gpu_pod(ctx, n, Bz, 1 - 1e-10, 8, prec=prec, valid=valid)
    Rn, mn, ln = _gpu_pod(ctx, n, Bn, 1 - 1e-10, 8, prec=prec, valid=valid)
    assert mn == mz and mz > 0
    assert np.array_equal(Rn, Rz)
    assert np.array_equal(ln, lz)
