"""Full-size and edge-case checks through the C ABI.

* 256^3 ABC (the mixed-precision workload's grid), FP64 and FP32 stencil, in
  a batch: oracle parity after two steps (the oracle finishes them in
  seconds), then over one whole 782-step subinterval the properties that
  hold at any size: sum conservation (FP64) and batch invariance.
* The 128^3 Kolmogorov solve in the benchmark's configuration, stopped after
  two iterations: the converged prefix is bitwise the GPU serial fine
  solution, ranks respect the caps, the report is consistent.
* Edge cases: N = 1 (no parareal subinterval: the solve is the warm-up fine
  solve), the smallest grid (n = 4), empty batches.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import fd
from gpu_helpers import rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_10981_amd as pr
    c = pr.Context(0)
    yield c
    c.close()


def test_fine_full_size_abc256(ctx):
    import torch
    import paper_2601_10981_amd as pr
    w = W.ABC_256_MIXED
    n = w.problem.n
    plan = pr.pr_plan(pr.problem_of(w.problem), w.opts)
    n_f, dt = plan["n_f"], plan["dt"]
    u0 = W.initial_field(w)
    p64 = pr.problem_of(dataclasses.replace(w.problem, precision=W.PREC_F64))
    p32 = pr.problem_of(w.problem)
    B = 3
    fields = [u0 * (1.0 - 0.2 * i) + 0.05 * i for i in range(B)]
    uin = torch.stack([to_dev(f) for f in fields])
    o64 = torch.empty_like(uin)
    o32 = torch.empty_like(uin)
    say("fine 256^3 x3, 2 steps, FP64 and FP32")
    for p, o in ((p64, o64), (p32, o32)):
        pr.pr_fine_propagate(ctx, [dict(prob=p, dt=dt, n_steps=2, u_in=uin[i], u_out=o[i])
                                   for i in range(B)])
    torch.cuda.synchronize()
    op = fd.Operator.of(w.problem)
    ref, _ = fd.fine_propagate(op, fields[B - 1], dt, 2)
    assert rel_l2(to_np(o64[B - 1]), ref) <= 1e-12
    assert rel_l2(to_np(o32[B - 1]), ref) <= 1e-5
    say(f"fine 256^3 x3, {n_f} steps, FP64")
    pr.pr_fine_propagate(ctx, [dict(prob=p64, dt=dt, n_steps=n_f, u_in=uin[i], u_out=o64[i])
                               for i in range(B)])
    torch.cuda.synchronize()
    s0, s1 = uin.sum(dim=1).cpu().numpy(), o64.sum(dim=1).cpu().numpy()
    a0 = uin.abs().sum(dim=1).cpu().numpy()
    assert np.all(np.abs(s1 - s0) <= 1e-11 * a0)
    one = torch.empty_like(uin[1])
    pr.pr_fine_propagate(ctx, [dict(prob=p64, dt=dt, n_steps=n_f, u_in=uin[1], u_out=one)])
    torch.cuda.synchronize()
    assert torch.equal(one, o64[1])


def test_solve_full_size_kolmogorov128_prefix(ctx):
    import torch
    import paper_2601_10981_amd as pr
    w = W.KOL_128_F64
    n, N = w.problem.n, w.opts.N
    p = pr.problem_of(w.problem)
    opts = dataclasses.replace(w.opts, max_iter=2)
    plan = pr.pr_plan(p, opts)
    u0 = to_dev(W.initial_field(w))
    ng = n ** 3
    say("solve 128^3, serial reference of 4 subintervals")
    ser = torch.empty((4, ng), dtype=torch.float64, device="cuda")
    ser[0].copy_(u0)
    for j in range(3):
        pr.pr_fine_propagate(ctx, [dict(prob=p, dt=plan["dt"], n_steps=plan["n_f"],
                                        u_in=ser[j], u_out=ser[j + 1])])
    say("solve 128^3, two iterations")
    U, rep = pr.pr_parareal_solve(ctx, p, opts, u0)
    torch.cuda.synchronize()
    assert rep.status == -5 and rep.iters == 2 and not rep.converged
    for j in range(4):                      # t = j DeltaT, j <= k + 1
        assert torch.equal(U[j], ser[j]), j
    assert rep.n_f == plan["n_f"] and rep.n_sub == N - 1 and rep.dM == plan["dM"]
    assert 1 <= rep.m0 <= opts.cap
    for k, row in enumerate(rep.ranks, start=1):
        assert len(row) == N - 1 - k and all(1 <= m <= opts.cap for m in row)
    assert all(np.isfinite(rep.jump)) and rep.jump[0] > 0
    assert rep.fine_updates == pytest.approx(
        (1 + (N - 1) + (N - 2)) * plan["n_f"] * ng, rel=1e-12)


def test_solve_single_subinterval(ctx):
    """N = 1: no parareal subinterval, the result is the fine solve of the
    warm-up window, converged at k = 0."""
    import torch
    import paper_2601_10981_amd as pr
    prob = W.Problem(n=12, kappa=0.1, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0))
    opts = W.PararealOpts(T=0.2, N=1, dt=0.01)
    u0 = W.blob_field(12, 3)
    p = pr.problem_of(prob)
    U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0))
    assert rep.iters == 0 and rep.converged and rep.status == 0
    n_f, dt = fd.steps_per_subinterval(opts.T, opts.dt)
    ref, _ = fd.fine_propagate(fd.Operator.of(prob), u0, dt, n_f)
    assert np.array_equal(to_np(U[0]), u0.reshape(-1))
    assert rel_l2(to_np(U[1]), ref) <= 1e-12


def test_smallest_grid_and_empty_batches(ctx):
    import torch
    import paper_2601_10981_amd as pr
    n = 4
    prob = W.Problem(n=n, kappa=0.05, flow=W.FLOW_ABC, fp=(1.0, 0.5, 0.25))
    p = pr.problem_of(prob)
    u0 = W.random_field(n, 9)
    u = to_dev(u0)
    out = torch.empty_like(u)
    pr.pr_fine_propagate(ctx, [dict(prob=p, dt=0.01, n_steps=7, u_in=u, u_out=out)])
    torch.cuda.synchronize()
    ref, _ = fd.fine_propagate(fd.Operator.of(prob), u0, 0.01, 7)
    assert rel_l2(to_np(out), ref) <= 1e-12
    # empty batches are no-ops
    pr.pr_fine_propagate(ctx, [])
    pr.pr_pod_build(ctx, [])
    pr.pr_coarse_propagate(ctx, [])
    assert pr.pr_solve_step_batch(ctx, []) == []


def test_forced_fine_full_size_paper_kolmogorov128(ctx):
    """The forced stencil at 128^3 in the launch shape the paper-flow bench
    times (40 fields, start times 5 (i + 1), delta t = 1e-2, kappa = 0.01):
    oracle parity after two steps, then over a whole 500-step subinterval
    the properties that hold at any size -- the grid sum is conserved (the
    Laplacian, the advection by a velocity whose components do not depend on
    their own coordinate, and the forcing, full periods of sin and cos, all
    sum to zero over the periodic grid) -- and batch invariance."""
    import torch
    import paper_2601_10981_amd as pr
    n, B, dt, kappa = 128, 40, 1e-2, 0.01
    prob = W.Problem(n=n, kappa=kappa, flow=W.FLOW_KOLMOGOROV_T, fp=(1.0, 1.0, 1.0))
    p = pr.problem_of(prob)
    fields = [W.fourier_field(n, 11 + i, n_modes=8, kmax=4.0) for i in (0, B - 1)]
    uin = torch.stack([to_dev(fields[0] if i < B - 1 else fields[1]) * (1.0 + 0.01 * i)
                       for i in range(B)])
    out = torch.empty_like(uin)
    items = [dict(prob=p, dt=dt, n_steps=2, u_in=uin[i], u_out=out[i], t0=5.0 * (i + 1))
             for i in range(B)]
    say("forced fine 128^3 x40, 2 steps")
    pr.pr_fine_propagate(ctx, items)
    torch.cuda.synchronize()
    op = fd.Operator.of(prob)
    for i in (0, B - 1):
        ref, _ = fd.fine_propagate(op, to_np(uin[i]).reshape(n, n, n), dt, 2, t0=5.0 * (i + 1))
        assert rel_l2(to_np(out[i]), ref) <= 1e-12, i
    say("forced fine 128^3 x40, 500 steps")
    for it in items:
        it["n_steps"] = 500
    pr.pr_fine_propagate(ctx, items)
    torch.cuda.synchronize()
    s0, s1 = uin.sum(dim=1).cpu().numpy(), out.sum(dim=1).cpu().numpy()
    a0 = uin.abs().sum(dim=1).cpu().numpy()
    assert np.all(np.abs(s1 - s0) <= 1e-10 * a0), np.max(np.abs(s1 - s0) / a0)
    one = torch.empty_like(uin[7])
    pr.pr_fine_propagate(ctx, [dict(prob=p, dt=dt, n_steps=500, u_in=uin[7], u_out=one,
                                    t0=5.0 * 8)])
    torch.cuda.synchronize()
    assert torch.equal(one, out[7])
