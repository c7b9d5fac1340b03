"""Incremental solves (pr_solve_begin / pr_solve_step_batch / pr_solve_end):
a solve advanced inside a mixed batch gives bitwise the iterates it gives
alone through pr_parareal_solve, whatever the batch holds (other grid sizes,
precisions, subinterval counts, modes, and steady or forced time-dependent
flows, whose fine solves then run as two launch groups); admission under a
budget; finished handles are left alone by later steps."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _case(n, N, prec, flow, fp, kappa, seed, tol=0.0, max_iter=0, cap0=6, cap=8,
          mode=W.MODE_ADAPTIVE):
    prob = W.Problem(n=n, kappa=kappa, flow=flow, fp=fp, precision=prec)
    opts = W.PararealOpts(T=0.1 * N, N=N, dt=0.01, cap0=cap0, cap=cap, tol=tol, max_iter=max_iter,
                          mode=mode)
    return prob, opts, W.fourier_field(n, seed, n_modes=6, kmax=3.0)


CASES = [
    _case(12, 8, W.PREC_F64, W.FLOW_KOLMOGOROV, (1.0, 2.0, 0.0), 0.1, 9),
    _case(16, 6, W.PREC_MIXED, W.FLOW_ABC, (1.0, 1.0, 1.0), 0.1, 5, tol=1e-6),
    _case(20, 10, W.PREC_F64, W.FLOW_ABC, (1.0, 0.7, 0.4), 0.05, 3, tol=1e-7, cap0=8, cap=10),
    _case(12, 5, W.PREC_F64, W.FLOW_UNIFORM, (1.0, 0.5, 0.25), 0.2, 11, max_iter=2),
    _case(16, 7, W.PREC_F64, W.FLOW_KOLMOGOROV, (1.0, 1.0, 0.0), 0.2, 13, tol=1e-8,
          mode=W.MODE_FIXED_POD),
    _case(16, 6, W.PREC_MIXED, W.FLOW_ABC, (1.0, 1.0, 1.0), 0.15, 14, tol=1e-7,
          mode=W.MODE_COARSE_GRID),
    _case(12, 6, W.PREC_F64, W.FLOW_KOLMOGOROV_T, (1.0, 1.0, 1.0), 0.1, 15),
    _case(16, 7, W.PREC_MIXED, W.FLOW_ABC_T, (1.0, 1.0, 1.0), 0.1, 16, tol=1e-7,
          mode=W.MODE_FIXED_POD),
]


def _gpu_serial(ctx, p, opts, u0):
    import torch
    import paper_2601_10981_amd as pr
    from oracle import fd
    n_f, dt = fd.steps_per_subinterval(opts.T / opts.N, opts.dt)
    ng = p.n ** 3
    out = torch.empty((opts.N + 1, ng), dtype=torch.float64, device="cuda")
    out[0].copy_(to_dev(u0))
    for j in range(opts.N):
        pr.pr_fine_propagate(ctx, [dict(prob=p, dt=dt, n_steps=n_f, u_in=out[j], u_out=out[j + 1],
                                        t0=j * opts.T / opts.N)])
    torch.cuda.synchronize()
    return out


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_10981_amd as pr
    c = pr.Context(0)
    yield c
    c.close()


def test_batched_solves_match_solo_bitwise(ctx):
    import paper_2601_10981_amd as pr
    solo = []
    for i, (prob, opts, u0) in enumerate(CASES):
        say(f"serving: solo solve {i} n={prob.n} N={opts.N} prec={prob.precision}")
        U, rep = pr.pr_parareal_solve(ctx, pr.problem_of(prob), opts, to_dev(u0))
        solo.append((to_np(U), rep))
    say("serving: batched")
    hs = [pr.pr_solve_begin(ctx, pr.problem_of(p), o, to_dev(u)) for p, o, u in CASES]
    assert all(h.nbytes > 0 for h in hs)
    steps = 0
    while not all(h.done for h in hs):
        flags = pr.pr_solve_step_batch(ctx, hs)
        assert flags == [h.done for h in hs]
        steps += 1
        assert steps <= max(o.N for _, o, _ in CASES)
    for i, h in enumerate(hs):
        U, rep = pr.pr_solve_end(ctx, h)
        Us, reps = solo[i]
        say(f"  solve {i}: iters {rep.iters} (solo {reps.iters}) status {rep.status}")
        assert rep.iters == reps.iters and rep.status == reps.status
        assert rep.converged == reps.converged and rep.m0 == reps.m0
        assert rep.ranks == reps.ranks
        assert rep.jump == reps.jump
        assert np.array_equal(to_np(U), Us), i


def test_staggered_arrivals_match_solo(ctx):
    """A solve admitted while others are mid-iteration (continuous batching)."""
    import paper_2601_10981_amd as pr
    (p0, o0, u0), (p1, o1, u1) = CASES[0], CASES[2]
    U0s = to_np(pr.pr_parareal_solve(ctx, pr.problem_of(p0), o0, to_dev(u0))[0])
    U1s = to_np(pr.pr_parareal_solve(ctx, pr.problem_of(p1), o1, to_dev(u1))[0])
    say("serving: staggered")
    a = pr.pr_solve_begin(ctx, pr.problem_of(p0), o0, to_dev(u0))
    pr.pr_solve_step_batch(ctx, [a])
    pr.pr_solve_step_batch(ctx, [a])
    b = pr.pr_solve_begin(ctx, pr.problem_of(p1), o1, to_dev(u1))
    live = [a, b]
    while live:
        pr.pr_solve_step_batch(ctx, live)
        live = [h for h in live if not h.done]
    Ua, ra = pr.pr_solve_end(ctx, a)
    Ub, rb = pr.pr_solve_end(ctx, b)
    Ua, Ub = to_np(Ua), to_np(Ub)
    say(f"  a: iters {ra.iters} status {ra.status}; b: iters {rb.iters} status {rb.status}")
    # a stops by finite termination (tol = 0): bitwise the serial fine solve
    assert ra.iters == o0.N - 1
    assert np.array_equal(Ua, to_np(_gpu_serial(ctx, pr.problem_of(p0), o0, u0)))
    assert np.array_equal(Ua, U0s)
    assert np.array_equal(Ub, U1s)


def test_finished_handle_untouched_and_budget_admission():
    import paper_2601_10981_amd as pr
    prob, opts, u0 = CASES[3]
    p = pr.problem_of(prob)
    need = pr.pr_footprint(p, opts)
    fixed_need = pr.pr_footprint(pr.problem_of(CASES[4][0]), CASES[4][1])
    assert 0 < fixed_need
    with pr.Context(0) as c:
        h = pr.pr_solve_begin(c, p, opts, to_dev(u0))
        while not h.done:
            pr.pr_solve_step_batch(c, [h])
        U1, r1 = pr.pr_solve_end(c, h)
        # a second handle: done handles are skipped by a step, and the
        # result does not change
        h = pr.pr_solve_begin(c, p, opts, to_dev(u0))
        while not h.done:
            pr.pr_solve_step_batch(c, [h])
        assert pr.pr_solve_step_batch(c, [h]) == [True]
        last = to_np(pr.pr_solve_state(c, h, opts.N))
        first = to_np(pr.pr_solve_state(c, h, 0))
        U2, r2 = pr.pr_solve_end(c, h)
        assert np.array_equal(last, to_np(U2[opts.N])) and np.array_equal(first, u0.reshape(-1))
        assert np.array_equal(to_np(U1), to_np(U2)) and r1.iters == r2.iters == 2
        assert r1.status == -5
    say(f"serving: admission, footprint {need} B")
    # a budget below one solve's minimum refuses it
    with pr.Context(0, budget_bytes=1 << 20) as c:
        with pytest.raises(pr.PrError) as e:
            pr.pr_solve_begin(c, p, opts, to_dev(u0))
        assert e.value.name == "PR_ENOMEM"
