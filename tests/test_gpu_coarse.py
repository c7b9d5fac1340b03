"""GPU parity of the coarse propagator (pr_coarse_propagate: eq. 8 / eq00,
augmentation eqaug / eq12 / eq13, reduced RK4) against the oracle, on the
same basis R fed to both sides."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import coarse, fd, pod
from gpu_helpers import rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_10981_amd as pr
    c = pr.Context(0)
    yield c
    c.close()


def _setup(n=12, cap=8, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0), kappa=0.05, seed=3):
    op = fd.Operator(n, kappa, flow, fp)
    h3 = op.h ** 3
    u0 = W.fourier_field(n, seed, n_modes=8, kmax=3.0)
    _, Wm = fd.fine_propagate(op, u0, 0.01, 30, 2)
    R, m, _ = pod.pod_mode(Wm, 1 - 5e-6, h3, cap)
    U1, _ = fd.fine_propagate(op, u0, 0.01, 40)
    U2 = U1 + 0.05 * W.random_field(n, seed + 7)
    return op, h3, R, m, U1.reshape(-1), U2.reshape(-1)


def _gpu(ctx, n, R, m, cap, u_in, dT, n_c, u_aug=None, prec=W.PREC_F64,
         flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0), kappa=0.05):
    import torch
    import paper_2601_10981_amd as pr
    fdt = torch.float32 if prec == W.PREC_MIXED else torch.float64
    prob = pr.problem(n, kappa, flow, fp, prec)
    Rp = np.zeros((n ** 3, cap))
    Rp[:, :R.shape[1]] = R
    dR = to_dev(Rp.T, fdt)
    dm = torch.tensor([m], dtype=torch.int32, device="cuda")
    ins = [to_dev(u) for u in u_in]
    outs = [torch.empty_like(x) for x in ins]
    beta = torch.zeros((len(ins), cap + 1), dtype=torch.float64, device="cuda")
    nco = torch.zeros(1, dtype=torch.int32, device="cuda")
    item = dict(prob=prob, R=dR, cap=cap, m=dm, u_in=ins, dT_total=dT, n_c=n_c, u_out=outs,
                beta_out=beta, n_c_out=nco)
    if u_aug is not None:
        item["u_aug"] = to_dev(u_aug)
    pr.pr_coarse_propagate(ctx, [item])
    torch.cuda.synchronize()
    return [to_np(o) for o in outs], to_np(beta), int(nco.item())


@pytest.mark.parametrize("cap,dT,n_c", [(8, 0.2, 5), (12, 0.5, 3), (31, 0.1, 2)])
def test_coarse_parity_augmented(ctx, cap, dT, n_c):
    say(f"coarse aug cap={cap}")
    op, h3, R, m, U1, U2 = _setup(cap=cap)
    Psi, aug = coarse.augment(R, U1, h3)
    assert aug
    lifted, betas, nc = coarse.coarse_propagate(op, Psi, [U1, U2], dT, n_c, h3)
    outs, beta, ncg = _gpu(ctx, op.n, R, m, cap, [U1, U2], dT, n_c, u_aug=U1)
    assert ncg == nc
    for o, l in zip(outs, lifted):
        assert rel_l2(o, l) <= 1e-12
    for i in range(2):
        bg = np.concatenate([beta[i, :m], beta[i, cap:cap + 1]])
        assert np.max(np.abs(bg - betas[i])) <= 1e-12 * np.max(np.abs(betas[i]))


def test_coarse_parity_plain(ctx):
    op, h3, R, m, U1, U2 = _setup(cap=10)
    lifted, betas, nc = coarse.coarse_propagate(op, R, [U2], 0.3, 4, h3)
    outs, beta, ncg = _gpu(ctx, op.n, R, m, 10, [U2], 0.3, 4)
    assert ncg == nc
    assert rel_l2(outs[0], lifted[0]) <= 1e-12


def test_coarse_guard_doubles_steps(ctx):
    op, h3, R, m, U1, U2 = _setup(cap=10)
    lifted, betas, nc = coarse.coarse_propagate(op, R, [U2], 5.0, 1, h3)
    assert nc > 1
    outs, beta, ncg = _gpu(ctx, op.n, R, m, 10, [U2], 5.0, 1)
    assert ncg == nc
    assert rel_l2(outs[0], lifted[0]) <= 1e-12


def test_coarse_state_in_span_skips_augmentation(ctx):
    op, h3, R, m, U1, U2 = _setup(cap=8)
    U = R @ np.linspace(1.0, 0.2, m)
    outs, beta, ncg = _gpu(ctx, op.n, R, m, 8, [U], 0.2, 3, u_aug=U)
    assert np.all(beta[0, 8] == 0.0)
    lifted, _, _ = coarse.coarse_propagate(op, R, [U], 0.2, 3, h3)
    assert rel_l2(outs[0], lifted[0]) <= 1e-12


def test_coarse_invariant_subspace_equals_fine(ctx):
    import torch
    import paper_2601_10981_amd as pr
    n, c, kappa = 16, (0.6, -0.9, 0.4), 0.05
    x = np.arange(n) * (2 * math.pi / n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    cols = []
    for k in [(1, 0, 0), (1, 2, -1), (0, 3, 1)]:
        a = k[0] * X + k[1] * Y + k[2] * Z
        cols += [np.cos(a).reshape(-1), np.sin(a).reshape(-1)]
    h3 = (2 * math.pi / n) ** 3
    Psi, kept = pod.m_orthonormalise(np.stack(cols, axis=1), h3)
    u0 = (0.7 * np.cos(X + 0.3) + 0.2 * np.sin(X + 2 * Y - Z) - 0.5 * np.cos(3 * Y + Z + 1.0))
    n_f, dt = 40, 0.01
    outs, _, _ = _gpu(ctx, n, Psi, 6, 6, [u0.reshape(-1)], n_f * dt, n_f,
                      flow=W.FLOW_UNIFORM, fp=c, kappa=kappa)
    prob = pr.problem(n, kappa, W.FLOW_UNIFORM, c)
    u = to_dev(u0)
    f = torch.empty_like(u)
    pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=dt, n_steps=n_f, u_in=u, u_out=f)])
    torch.cuda.synchronize()
    assert rel_l2(outs[0], to_np(f)) <= 1e-13


def test_coarse_mixed_precision(ctx):
    op, h3, R, m, U1, U2 = _setup(cap=8)
    Psi, aug = coarse.augment(R, U1, h3)
    lifted, betas, nc = coarse.coarse_propagate(op, Psi, [U1, U2], 0.2, 4, h3)
    outs, beta, ncg = _gpu(ctx, op.n, R, m, 8, [U1, U2], 0.2, 4, u_aug=U1, prec=W.PREC_MIXED)
    for o, l in zip(outs, lifted):
        assert rel_l2(o, l) <= 1e-5


@pytest.mark.parametrize("prec", [W.PREC_F64, W.PREC_MIXED], ids=["f64", "mixed"])
def test_coarse_rank_zero_basis_augments_by_u(ctx, prec):
    """A basis of rank 0 (every column masked): both Gram-Schmidt passes
    leave u unchanged, so the coarse space is span{u} and the propagation
    is the scalar reduced system of that one column."""
    say(f"coarse rank-0 basis prec={prec}")
    cap = 8
    op, h3, R, m, U1, U2 = _setup(cap=cap)
    R0 = np.zeros((op.n ** 3, 0))
    Psi, aug = coarse.augment(R0, U1, h3)
    assert aug and Psi.shape[1] == 1
    lifted, betas, nc = coarse.coarse_propagate(op, Psi, [U1, U2], 0.2, 4, h3)
    # garbage in the masked columns must not leak into the result
    Rg = np.full((op.n ** 3, cap), np.nan)
    outs, beta, ncg = _gpu(ctx, op.n, Rg, 0, cap, [U1, U2], 0.2, 4, u_aug=U1, prec=prec)
    assert ncg == nc
    tol = 1e-12 if prec == W.PREC_F64 else 1e-6
    for o, l in zip(outs, lifted):
        assert np.all(np.isfinite(o))
        assert rel_l2(o, l) <= tol
    for i in range(2):
        assert abs(beta[i, cap] - betas[i][0]) <= tol * abs(betas[i][0])
        assert np.all(beta[i, :cap] == 0.0)


@pytest.mark.parametrize("n,flow,fp,prec", [
    (64, W.FLOW_ABC, (1.0, 1.0, 1.0), W.PREC_F64),
    (72, W.FLOW_ABC, (0.8, 1.1, 0.6), W.PREC_F64),
    (72, W.FLOW_KOLMOGOROV, (0.8, 3.0, 0.0), W.PREC_F64),
    (72, W.FLOW_ABC, (1.0, 1.0, 1.0), W.PREC_MIXED)],
    ids=["abc64", "abc72", "kol72", "abc72_mixed"])
def test_coarse_L_window_kernel(ctx, monkeypatch, n, flow, fp, prec):
    """L applied through the LDS window of each plane (the kernel the solver
    uses for the bases of many subintervals at 64^3 and up): bitwise the
    per-column kernel's L Psi, hence the same coarse outputs, on grids whose
    plane is not a whole number of windows (72^2 = 5.06 x 1024), and the
    oracle's values in FP64 (1e-12)."""
    say(f"coarse L window kernel n={n} flow={flow} prec={prec}")
    cap = 8
    op, h3, R, m, U1, U2 = _setup(n=n, cap=cap, flow=flow, fp=fp)
    res = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("PR_APPLYL_WIN", mode)
        res[mode] = _gpu(ctx, n, R, m, cap, [U1, U2], 0.2, 3, u_aug=U1, prec=prec,
                         flow=flow, fp=fp)
    monkeypatch.delenv("PR_APPLYL_WIN")
    for a, b in zip(res["0"][0], res["1"][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(res["0"][1], res["1"][1])
    if prec == W.PREC_F64:
        Psi, aug = coarse.augment(R, U1, h3)
        lifted, _, _ = coarse.coarse_propagate(op, Psi, [U1, U2], 0.2, 3, h3)
        for o, l in zip(res["1"][0], lifted):
            assert rel_l2(o, l) <= 1e-12


@pytest.mark.parametrize("n,prec", [(256, W.PREC_F64), (250, W.PREC_MIXED)],
                         ids=["n256_f64", "n250_mixed"])
def test_coarse_L_window_kernel_largest_grids(ctx, monkeypatch, n, prec):
    """The window kernel at the top of its range (n = 256: a 1536-value window
    per plane) and on a plane of 62,500 points (61.04 windows): the coarse
    outputs are bitwise those of the per-column kernel. A random
    M-orthonormal basis stands in for a POD basis (no oracle at this size)."""
    say(f"coarse L window kernel n={n} prec={prec}")
    rng = np.random.default_rng(11)
    cap, m = 8, 6
    h3 = (2 * math.pi / n) ** 3
    Q, _ = np.linalg.qr(rng.standard_normal((n ** 3, m)))
    R = Q / math.sqrt(h3)
    U1 = rng.standard_normal(n ** 3)
    U2 = U1 + 0.1 * rng.standard_normal(n ** 3)
    res = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("PR_APPLYL_WIN", mode)
        res[mode] = _gpu(ctx, n, R, m, cap, [U1, U2], 0.05, 2, u_aug=U1, prec=prec)
    monkeypatch.delenv("PR_APPLYL_WIN")
    for a, b in zip(res["0"][0], res["1"][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(res["0"][1], res["1"][1])
    assert np.all(np.isfinite(res["1"][1]))
