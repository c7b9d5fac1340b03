"""GPU parity of the fine propagator (pr_fine_propagate) against the oracle.

FP64: relative L2 <= 1e-12 per field and per snapshot; FP32 stencil (mixed):
<= 1e-5. Shapes span several tiles with ragged tails (n = 20 leaves partial
(y, z) tiles and, at 16-plane chunks, an x split 16 + 4; n = 33 is odd).
Batches mix sizes, flows, steps and dt in one launch.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fd
from gpu_helpers import rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu

CASES = [
    # n, flow, fp, kappa, dt, steps, snap_every, seed
    (16, W.FLOW_ABC, (1.0, 1.0, 1.0), 0.05, 0.01, 7, 2, 1),
    (20, W.FLOW_KOLMOGOROV, (1.0, 2.0, 0.0), 0.03, 0.02, 5, 5, 2),
    (33, W.FLOW_ABC, (1.0, 0.5, 0.3), 0.1, 0.004, 4, 1, 3),
    (32, W.FLOW_UNIFORM, (0.3, -0.7, 1.1), 0.02, 0.01, 6, 3, 4),
]


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_10981_amd as pr
    c = pr.Context(0)
    yield c
    c.close()


def _prob(n, flow, fp, kappa, prec=W.PREC_F64):
    import paper_2601_10981_amd as pr
    return pr.problem(n, kappa, flow, fp, prec)


def _oracle(n, flow, fp, kappa, dt, steps, se, u0):
    op = fd.Operator(n, kappa, flow, fp)
    out, Wm = fd.fine_propagate(op, u0, dt, steps, se)
    return out.reshape(-1), Wm


def _run(ctx, cases, prec=W.PREC_F64):
    import torch
    import paper_2601_10981_amd as pr
    items, outs, snaps = [], [], []
    fdt = torch.float32 if prec == W.PREC_MIXED else torch.float64
    for (n, flow, fp, kappa, dt, steps, se, seed) in cases:
        u0 = W.random_field(n, seed)
        uin = to_dev(u0)
        uout = torch.empty_like(uin)
        sn = torch.empty((steps // se + 1, n ** 3), dtype=fdt, device="cuda")
        items.append(dict(prob=_prob(n, flow, fp, kappa, prec), dt=dt, n_steps=steps, u_in=uin,
                          u_out=uout, snap_every=se, snaps=sn))
        outs.append(uout)
        snaps.append(sn)
    pr.pr_fine_propagate(ctx, items)
    torch.cuda.synchronize()
    return outs, snaps


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}-flow{c[1]}")
def test_fine_parity_f64(ctx, case):
    say(f"fine parity f64 {case}")
    outs, snaps = _run(ctx, [case])
    n, flow, fp, kappa, dt, steps, se, seed = case
    ref, Wm = _oracle(n, flow, fp, kappa, dt, steps, se, W.random_field(n, seed))
    assert rel_l2(to_np(outs[0]), ref) <= 1e-12
    S = to_np(snaps[0]).reshape(-1, n ** 3)
    assert S.shape[0] == Wm.shape[1]
    for j in range(S.shape[0]):
        assert rel_l2(S[j], Wm[:, j]) <= 1e-12, j


def test_fine_batch_uneven_is_bitwise_batch_invariant(ctx):
    say("fine batch uneven")
    outs_b, snaps_b = _run(ctx, CASES)
    for i, case in enumerate(CASES):
        outs_1, snaps_1 = _run(ctx, [case])
        assert np.array_equal(to_np(outs_b[i]), to_np(outs_1[0])), case
        assert np.array_equal(to_np(snaps_b[i]), to_np(snaps_1[0])), case
        n, flow, fp, kappa, dt, steps, se, seed = case
        ref, _ = _oracle(n, flow, fp, kappa, dt, steps, se, W.random_field(n, seed))
        assert rel_l2(to_np(outs_b[i]), ref) <= 1e-12


@pytest.mark.parametrize("prec", [W.PREC_F64, W.PREC_MIXED], ids=["f64", "mixed"])
def test_fine_every_tile_configuration_is_bitwise_identical(ctx, prec, monkeypatch):
    """Each point's arithmetic is independent of the tiling and of the x-chunk
    length, so every launch shape the autotuner may pick gives the same bits
    (the first batch of each key also runs the tuner itself)."""
    say(f"fine tile configurations prec={prec}")
    cases = CASES + [(40, W.FLOW_ABC, (1.0, 1.0, 1.0), 0.05, 0.005, 3, 1, 6)]
    ref_outs, ref_snaps = _run(ctx, cases, prec)          # autotuned
    for pol in range(3):
        monkeypatch.setenv("PR_FUSED_CHUNK", str(pol))
        for cfg in range(11):   # the blocked tilings 8..10 fall back (n = 33 is odd)
            monkeypatch.setenv("PR_FUSED_CFG", str(cfg))
            outs, snaps = _run(ctx, cases, prec)
            for i in range(len(cases)):
                assert np.array_equal(to_np(outs[i]), to_np(ref_outs[i])), (pol, cfg, i)
                assert np.array_equal(to_np(snaps[i]), to_np(ref_snaps[i])), (pol, cfg, i)
    monkeypatch.delenv("PR_FUSED_CFG")
    monkeypatch.delenv("PR_FUSED_CHUNK")


EVEN_CASES = [c for c in CASES if c[0] % 2 == 0] + [
    (40, W.FLOW_ABC, (1.0, 1.0, 1.0), 0.05, 0.005, 3, 1, 6),
    (36, W.FLOW_KOLMOGOROV, (0.8, 3.0, 0.0), 0.02, 0.01, 7, 3, 7)]


@pytest.mark.parametrize("prec", [W.PREC_F64, W.PREC_MIXED], ids=["f64", "mixed"])
def test_fine_blocked_tilings_are_bitwise_the_column_ones(ctx, prec, monkeypatch):
    """The 2 x 2 register-blocked tilings (each thread four columns, LDS in
    even/odd-z sub-planes) compute every point with the same operations as
    the one-column tilings: bitwise the same fields and snapshots under every
    chunk policy, on even grids with ragged tiles (n = 20, 36, 40 against
    32 x 32 and 16 x 64 tiles), and the oracle's values (FP64 1e-12)."""
    import paper_2601_10981_amd as pr
    say(f"fine blocked tilings prec={prec}")
    monkeypatch.setenv("PR_FUSED_CFG", "0")
    ref_outs, ref_snaps = _run(ctx, EVEN_CASES, prec)
    for pol in range(3):
        monkeypatch.setenv("PR_FUSED_CHUNK", str(pol))
        for cfg in (8, 9, 10):
            monkeypatch.setenv("PR_FUSED_CFG", str(cfg))
            outs, snaps = _run(ctx, EVEN_CASES, prec)
            t = pr.pr_fine_tuned(ctx, prec, 40, len(EVEN_CASES), blocked=True)
            assert t[3] == 1, t
            for i in range(len(EVEN_CASES)):
                assert np.array_equal(to_np(outs[i]), to_np(ref_outs[i])), (pol, cfg, i)
                assert np.array_equal(to_np(snaps[i]), to_np(ref_snaps[i])), (pol, cfg, i)
    monkeypatch.delenv("PR_FUSED_CFG")
    monkeypatch.delenv("PR_FUSED_CHUNK")
    if prec == W.PREC_F64:
        for i, case in enumerate(EVEN_CASES):
            n, flow, fp, kappa, dt, steps, se, seed = case
            ref, _ = _oracle(n, flow, fp, kappa, dt, steps, se, W.random_field(n, seed))
            assert rel_l2(to_np(ref_outs[i]), ref) <= 1e-12, case


def test_fine_run_to_run_bitwise(ctx):
    a, _ = _run(ctx, CASES[:2])
    b, _ = _run(ctx, CASES[:2])
    for x, y in zip(a, b):
        assert np.array_equal(to_np(x), to_np(y))


def test_fine_in_place(ctx):
    import torch
    import paper_2601_10981_amd as pr
    n, flow, fp, kappa, dt, steps, se, seed = CASES[0]
    u = to_dev(W.random_field(n, seed))
    pr.pr_fine_propagate(ctx, [dict(prob=_prob(n, flow, fp, kappa), dt=dt, n_steps=steps,
                                    u_in=u, u_out=u)])
    torch.cuda.synchronize()
    ref, _ = _oracle(n, flow, fp, kappa, dt, steps, se, W.random_field(n, seed))
    assert rel_l2(to_np(u), ref) <= 1e-12


@pytest.mark.parametrize("case", CASES[:3], ids=lambda c: f"n{c[0]}")
def test_fine_mixed_precision(ctx, case):
    say(f"fine mixed {case}")
    outs, snaps = _run(ctx, [case], prec=W.PREC_MIXED)
    n, flow, fp, kappa, dt, steps, se, seed = case
    ref, Wm = _oracle(n, flow, fp, kappa, dt, steps, se, W.random_field(n, seed))
    assert rel_l2(to_np(outs[0]), ref) <= 1e-5
    S = to_np(snaps[0]).reshape(-1, n ** 3)
    for j in range(S.shape[0]):
        assert rel_l2(S[j], Wm[:, j]) <= 1e-5


def test_fine_fourier_mode_closed_form(ctx):
    import torch
    import paper_2601_10981_amd as pr
    n, kappa, c = 24, 0.03, (0.7, -0.4, 1.1)
    k = (1, 2, -3)
    x = np.arange(n) * (2 * math.pi / n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    arg = k[0] * X + k[1] * Y + k[2] * Z
    h = 2 * math.pi / n
    lam = -(4 * kappa / h ** 2) * sum(math.sin(kd * h / 2) ** 2 for kd in k) \
        - 1j * sum(cd * math.sin(kd * h) / h for kd, cd in zip(k, c))
    dt, steps = 0.3 / abs(lam), 11
    z = dt * lam
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    exact = abs(R) ** steps * np.cos(arg + steps * np.angle(R))
    u = to_dev(np.cos(arg))
    out = torch.empty_like(u)
    pr.pr_fine_propagate(ctx, [dict(prob=_prob(n, W.FLOW_UNIFORM, c, kappa), dt=dt,
                                    n_steps=steps, u_in=u, u_out=out)])
    torch.cuda.synchronize()
    assert np.max(np.abs(to_np(out) - exact.reshape(-1))) <= 1e-13


def test_fine_errors(ctx):
    import torch
    import paper_2601_10981_amd as pr
    u = to_dev(W.random_field(16, 1))
    out = torch.empty_like(u)
    with pytest.raises(pr.PrError) as e:
        pr.pr_fine_propagate(ctx, [dict(prob=_prob(16, W.FLOW_ABC, (1, 1, 1), 0.05), dt=1.0,
                                        n_steps=1, u_in=u, u_out=out)])
    assert e.value.name == "PR_EUNSTABLE"
    with pytest.raises(pr.PrError) as e:
        pr.pr_fine_propagate(ctx, [dict(prob=_prob(16, W.FLOW_ABC, (1, 1, 1), 0.05), dt=-1.0,
                                        n_steps=1, u_in=u, u_out=out)])
    assert e.value.name == "PR_EINVAL"
    # zero steps copies
    pr.pr_fine_propagate(ctx, [dict(prob=_prob(16, W.FLOW_ABC, (1, 1, 1), 0.05), dt=0.01,
                                    n_steps=0, u_in=u, u_out=out)])
    torch.cuda.synchronize()
    assert np.array_equal(to_np(out), to_np(u))


def test_fine_full_size_kolmogorov128(ctx):
    """The 128^3 Kolmogorov workload in the launch shape the benchmark uses (a
    batch of subinterval fields): sampled oracle parity on two fields after
    three steps, and exact sum conservation plus batch invariance over the
    full 157-step subinterval on the whole batch."""
    import torch
    import paper_2601_10981_amd as pr
    w = W.KOL_128_F64
    n = w.problem.n
    prob = pr.problem_of(w.problem)
    u0 = W.initial_field(w)
    n_f, dt = fd.steps_per_subinterval(w.opts.T / w.opts.N, w.opts.dt)
    B = 16
    fields = [u0 * (1.0 + 0.1 * i) + 0.01 * i for i in range(B)]
    uin = torch.stack([to_dev(f) for f in fields])
    uout = torch.empty_like(uin)
    say("fine 128^3 x16, 3 steps")
    pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=dt, n_steps=3, u_in=uin[i], u_out=uout[i])
                               for i in range(B)])
    torch.cuda.synchronize()
    op = fd.Operator.of(w.problem)
    for i in (0, B - 1):
        ref, _ = fd.fine_propagate(op, fields[i], dt, 3)
        assert rel_l2(to_np(uout[i]), ref) <= 1e-12
    say(f"fine 128^3 x16, {n_f} steps")
    pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=dt, n_steps=n_f, u_in=uin[i], u_out=uout[i])
                               for i in range(B)])
    torch.cuda.synchronize()
    s0 = uin.sum(dim=1).cpu().numpy()
    s1 = uout.sum(dim=1).cpu().numpy()
    a0 = uin.abs().sum(dim=1).cpu().numpy()
    assert np.all(np.abs(s1 - s0) <= 1e-11 * a0)
    one = torch.empty_like(uin[3])
    pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=dt, n_steps=n_f, u_in=uin[3], u_out=one)])
    torch.cuda.synchronize()
    assert torch.equal(one, uout[3])


@pytest.mark.parametrize("forced_cfg", [None, "8"], ids=["tuned", "b22_32x32"])
def test_fine_full_size_bench_launch_63_fields(ctx, monkeypatch, forced_cfg):
    """The stencil launch the benchmark times: 63 subinterval fields of the
    128^3 Kolmogorov workload in one batched launch (the autotuner's pick,
    and the 2 x 2 blocked 32 x 32 tiling over whole 128-plane chunks that
    the committed profile covers). Sampled oracle parity on the first, a
    middle and the last field after three steps (<= 1e-12), and bitwise
    agreement of every field with the same field propagated alone."""
    import torch
    import paper_2601_10981_amd as pr
    if forced_cfg is not None:
        monkeypatch.setenv("PR_FUSED_CFG", forced_cfg)
        monkeypatch.setenv("PR_FUSED_CHUNK", "1")
    w = W.KOL_128_F64
    prob = pr.problem_of(w.problem)
    u0 = to_dev(W.initial_field(w))
    n_f, dt = fd.steps_per_subinterval(w.opts.T / w.opts.N, w.opts.dt)
    B = w.opts.N - 1
    uin = torch.stack([u0 * (1.0 + 0.01 * i) for i in range(B)])
    uout = torch.empty_like(uin)
    say(f"fine 128^3 x{B}, 3 steps, cfg {forced_cfg}")
    pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=dt, n_steps=3, u_in=uin[i], u_out=uout[i])
                               for i in range(B)])
    torch.cuda.synchronize()
    if forced_cfg is not None:
        t = pr.pr_fine_tuned(ctx, pr.PR_F64, w.problem.n, B, planes=True, blocked=True)
        assert t == (32, 32, 448, 128, 1), t
    op = fd.Operator.of(w.problem)
    for i in (0, B // 2, B - 1):
        n = w.problem.n
        ref, _ = fd.fine_propagate(op, to_np(uin[i]).reshape(n, n, n), dt, 3)
        assert rel_l2(to_np(uout[i]), ref) <= 1e-12, i
    one = torch.empty_like(uin[0])
    for i in (0, B - 1):
        pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=dt, n_steps=3, u_in=uin[i], u_out=one)])
        torch.cuda.synchronize()
        assert torch.equal(one, uout[i]), i
