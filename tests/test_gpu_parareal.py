"""GPU parity of the whole adaptive parareal solve (pr_parareal_solve,
formula4 / Algorithm 2) against the oracle.

* finite termination: after N - 1 iterations the GPU result equals the GPU
  serial fine solve bitwise (same kernels) and the oracle's serial solve to
  1e-12;
* the converged prefix U^k_j, j <= k, equals the serial fine solve bitwise;
* iterate by iterate (max_iter = k stops after k iterations and returns the
  iterate) against the oracle, with identical stage-2 ranks;
* the 32^3 ABC workload end to end.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fd, parareal
from gpu_helpers import rel_l2, roundoff_envelope as _roundoff_envelope, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_10981_amd as pr
    c = pr.Context(0)
    yield c
    c.close()


def gpu_serial(ctx, prob, opts, u0):
    """Serial fine solution on the GPU at t = j DeltaT (N + 1 fields)."""
    import torch
    import paper_2601_10981_amd as pr
    n_f, dt = fd.steps_per_subinterval(opts.T / opts.N, opts.dt)
    ng = prob.n ** 3
    out = torch.empty((opts.N + 1, ng), dtype=torch.float64, device="cuda")
    out[0].copy_(to_dev(u0))
    for j in range(opts.N):
        pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=dt, n_steps=n_f, u_in=out[j], u_out=out[j + 1])])
    torch.cuda.synchronize()
    return out


def _tiny(n=12, N=6, T=0.6, tol=0.0, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0), kappa=0.05,
          cap0=6, cap=8, max_iter=0, prec=W.PREC_F64):
    prob = W.Problem(n=n, kappa=kappa, flow=flow, fp=fp, precision=prec)
    opts = W.PararealOpts(T=T, N=N, dt=0.01, cap0=cap0, cap=cap, tol=tol, max_iter=max_iter)
    return prob, opts


def test_parareal_finite_termination(ctx):
    import paper_2601_10981_amd as pr
    say("parareal finite termination")
    prob, opts = _tiny()
    u0 = W.blob_field(prob.n, 7)
    p = pr.problem_of(prob)
    ref = gpu_serial(ctx, p, opts, u0)
    U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=ref)
    assert rep.iters == opts.N - 1 and rep.converged
    assert np.array_equal(to_np(U), to_np(ref))
    oref = parareal.reference(prob, opts, u0)
    for j in range(opts.N + 1):
        assert rel_l2(to_np(U[j]), oref[j]) <= 1e-12
    assert rep.err[-1] == 0.0


@pytest.mark.parametrize("ml,p", [(1, 1), (0, 0), (1, 0), (0, 1)])
def test_parareal_prefix_and_iterates_match_oracle(ctx, ml, p):
    """Iterates of every local-in-time collection (m_l, p) in {0,1}^2 (the
    grid of the paper's experiments) against the oracle."""
    import paper_2601_10981_amd as pr
    prob, opts = _tiny(n=12, N=8, T=0.8, kappa=0.1, flow=W.FLOW_KOLMOGOROV, fp=(1.0, 2.0, 0.0))
    opts = W.PararealOpts(**{**opts.__dict__, "ml": ml, "p": p})
    u0 = W.fourier_field(prob.n, 9, n_modes=6, kmax=3.0)
    p = pr.problem_of(prob)
    ref = gpu_serial(ctx, p, opts, u0)
    ores = parareal.solve(prob, opts, u0, keep_history=True)
    env = _roundoff_envelope(prob, opts, u0, ores, 3)
    for k in range(1, 4):
        say(f"parareal iterate k={k} (m_l, p) = ({ml}, {p})")
        o = W.PararealOpts(**{**opts.__dict__, "max_iter": k})
        U, rep = pr.pr_parareal_solve(ctx, p, o, to_dev(u0), U_ref=ref)
        assert rep.iters == k
        Un = to_np(U)
        # converged prefix: time index j + 1 <= k + 1 equals the serial solve bitwise
        for j in range(0, k + 2):
            assert np.array_equal(Un[j], to_np(ref[j])), (k, j)
        # stage-2 ranks are identical to the oracle's
        assert rep.ranks[k - 1] == ores.ranks[k], (k, rep.ranks[k - 1], ores.ranks[k])
        hist = ores.history[k]
        worst = max(rel_l2(Un[j + 1], hist[j]) for j in range(len(hist)))
        say(f"  k={k} worst iterate rel L2 vs oracle {worst:.3e} (round-off envelope {env[k]:.3e})")
        assert worst <= 10.0 * env[k] + 1e-12


def test_parareal_iterates_at_1e12_on_a_well_separated_spectrum(ctx):
    """Iterates k = 1..3 of (m_l, p) = (1, 1) in FP64 held to 1e-12 against
    the oracle. The rank caps cut every POD spectrum of this case at a wide
    gap (lambda_{m+1} / lambda_m <= 0.32), so the kept subspaces are fixed by
    the data to round-off: the oracle's own one-ulp perturbation envelope
    stays below 1e-13, and the GPU must agree to 1e-12."""
    import paper_2601_10981_amd as pr
    prob, opts = _tiny(n=12, N=8, T=0.8, kappa=0.1, flow=W.FLOW_KOLMOGOROV, fp=(1.0, 2.0, 0.0),
                       cap0=3, cap=4)
    u0 = W.fourier_field(prob.n, 9, n_modes=6, kmax=3.0)
    p = pr.problem_of(prob)
    ref = gpu_serial(ctx, p, opts, u0)
    o3 = W.PararealOpts(**{**opts.__dict__, "max_iter": 3})
    ores = parareal.solve(prob, o3, u0, keep_history=True)
    env = _roundoff_envelope(prob, o3, u0, ores, 3)
    say(f"well-separated case: oracle round-off envelope {['%.1e' % e for e in env[1:]]}")
    assert max(env[1:]) <= 1e-13
    for k in range(1, 4):
        o = W.PararealOpts(**{**opts.__dict__, "max_iter": k})
        U, rep = pr.pr_parareal_solve(ctx, p, o, to_dev(u0), U_ref=ref)
        assert rep.iters == k
        assert rep.ranks[k - 1] == ores.ranks[k]
        Un = to_np(U)
        worst = max(rel_l2(Un[j + 1], ores.history[k][j]) for j in range(len(ores.history[k])))
        say(f"  k={k} worst iterate rel L2 vs oracle {worst:.3e}")
        assert worst <= 1e-12


def test_parareal_abc32_workload(ctx):
    """The 32^3 ABC FP64 workload end to end against the oracle."""
    import paper_2601_10981_amd as pr
    w = W.ABC_32_F64
    u0 = W.initial_field(w)
    p = pr.problem_of(w.problem)
    say("parareal abc32: oracle")
    oref = parareal.reference(w.problem, w.opts, u0)
    ores = parareal.solve(w.problem, w.opts, u0, U_ref=oref)
    say("parareal abc32: gpu")
    ref = gpu_serial(ctx, p, w.opts, u0)
    for j in range(w.opts.N + 1):
        assert rel_l2(to_np(ref[j]), oref[j]) <= 1e-12
    U, rep = pr.pr_parareal_solve(ctx, p, w.opts, to_dev(u0), U_ref=ref)
    say(f"  iters gpu {rep.iters} oracle {ores.iters}; errs gpu {rep.err} oracle {ores.errors}")
    assert rep.iters == ores.iters
    assert rep.m0 == ores.m0
    for j in range(w.opts.N + 1):
        assert rel_l2(to_np(U[j]), ores.U[j]) <= 1e-12
    for eg, eo in zip(rep.err, ores.errors):
        assert abs(eg - eo) <= 1e-6 * max(eo, 1e-12) + 1e-12
    for k in range(1, rep.iters + 1):
        assert rep.ranks[k - 1] == ores.ranks[k]


def test_parareal_converges_before_finite_termination(ctx):
    import paper_2601_10981_amd as pr
    prob, opts = _tiny(n=12, N=12, T=1.2, kappa=0.3, tol=1e-7, flow=W.FLOW_KOLMOGOROV,
                       fp=(1.0, 2.0, 0.0), cap0=8, cap=12)
    u0 = W.fourier_field(prob.n, 9, n_modes=6, kmax=3.0)
    p = pr.problem_of(prob)
    ref = gpu_serial(ctx, p, opts, u0)
    ores = parareal.solve(prob, opts, u0)
    U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=ref)
    say(f"converging: gpu iters {rep.iters} jumps {rep.jump}; oracle {ores.iters} {ores.jumps}")
    assert rep.converged and rep.iters == ores.iters < opts.N - 1
    assert rep.err[-1] <= 1e-6
    for j in range(opts.N + 1):
        assert rel_l2(to_np(U[j]), ores.U[j]) <= 1e-9


def test_parareal_mixed_precision_converges(ctx):
    import paper_2601_10981_amd as pr
    prob, opts = _tiny(n=16, N=8, T=0.8, kappa=0.1, tol=1e-6, prec=W.PREC_MIXED, cap0=8, cap=12)
    u0 = W.fourier_field(prob.n, 5, n_modes=8, kmax=4.0)
    p64 = pr.problem_of(W.Problem(n=16, kappa=0.1, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0)))
    ref = gpu_serial(ctx, p64, opts, u0)
    U, rep = pr.pr_parareal_solve(ctx, pr.problem_of(prob), opts, to_dev(u0), U_ref=ref)
    say(f"mixed: iters {rep.iters} errs {rep.err}")
    assert rep.err[-1] <= 1e-5
    oref = parareal.reference(W.Problem(n=16, kappa=0.1, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0)),
                              opts, u0)
    assert rel_l2(to_np(U[-1]), oref[-1]) <= 1e-5


def test_parareal_errors(ctx):
    import paper_2601_10981_amd as pr
    prob, opts = _tiny()
    p = pr.problem_of(prob)
    u0 = to_dev(W.blob_field(prob.n, 1))
    # DeltaT = 1 with dt = 1: dt * rho(L) ~ 13.6 > 2.6
    bad = W.PararealOpts(**{**opts.__dict__, "dt": 1.0, "T": 6.0})
    with pytest.raises(pr.PrError) as e:
        pr.pr_parareal_solve(ctx, p, bad, u0)
    assert e.value.name == "PR_EUNSTABLE"
    bad = W.PararealOpts(**{**opts.__dict__, "cap": 40})
    with pytest.raises(pr.PrError) as e:
        pr.pr_parareal_solve(ctx, p, bad, u0)
    assert e.value.name == "PR_EINVAL"
    one = W.PararealOpts(**{**opts.__dict__, "max_iter": 1, "tol": 0.0})
    U, rep = pr.pr_parareal_solve(ctx, p, one, u0)
    assert rep.status == -5 and rep.iters == 1


def test_fixed_pod_mode_matches_oracle(ctx):
    """The fixed-POD comparison method ("Parareal-I", Sec. 4): iterates
    against the oracle within its round-off envelope, finite termination
    bitwise against the GPU serial solve, and the same k = 0 step as the
    adaptive mode."""
    import paper_2601_10981_amd as pr
    prob, opts = _tiny(n=12, N=8, T=0.8, kappa=0.1, flow=W.FLOW_KOLMOGOROV, fp=(1.0, 2.0, 0.0))
    opts = W.PararealOpts(**{**opts.__dict__, "mode": W.MODE_FIXED_POD})
    u0 = W.fourier_field(prob.n, 9, n_modes=6, kmax=3.0)
    p = pr.problem_of(prob)
    ref = gpu_serial(ctx, p, opts, u0)
    ores = parareal.solve(prob, opts, u0, keep_history=True)
    env = _roundoff_envelope(prob, opts, u0, ores, 3)
    for k in range(1, 4):
        say(f"fixed-POD iterate k={k}")
        o = W.PararealOpts(**{**opts.__dict__, "max_iter": k})
        U, rep = pr.pr_parareal_solve(ctx, p, o, to_dev(u0), U_ref=ref)
        assert rep.iters == k and rep.m0 == ores.m0
        Un = to_np(U)
        for j in range(0, k + 2):
            assert np.array_equal(Un[j], to_np(ref[j])), (k, j)
        worst = max(rel_l2(Un[j + 1], h) for j, h in enumerate(ores.history[k]))
        say(f"  k={k} worst rel L2 vs oracle {worst:.3e} (envelope {env[k]:.3e})")
        assert worst <= 10.0 * env[k] + 1e-12
    U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=ref)
    assert rep.iters == opts.N - 1 and rep.converged
    assert np.array_equal(to_np(U), to_np(ref))
    # k = 0 is the adaptive method's
    a0 = W.PararealOpts(**{**opts.__dict__, "mode": W.MODE_ADAPTIVE, "max_iter": 1})
    f0 = W.PararealOpts(**{**opts.__dict__, "max_iter": 1})
    _, ra = pr.pr_parareal_solve(ctx, p, a0, to_dev(u0), U_ref=ref)
    _, rf = pr.pr_parareal_solve(ctx, p, f0, to_dev(u0), U_ref=ref)
    assert ra.err[0] == rf.err[0] and ra.m0 == rf.m0


@pytest.mark.parametrize("prec", [W.PREC_F64, W.PREC_MIXED], ids=["f64", "mixed"])
def test_coarse_grid_mode_matches_oracle(ctx, prec):
    """The coarse-grid comparison method ("Parareal-II", Sec. 4): no POD, so
    FP64 iterates match the oracle to 1e-12 at every k (mixed precision: the
    FP32 stencil's 1e-5); finite termination bitwise against the GPU serial
    solve (FP64)."""
    import paper_2601_10981_amd as pr
    prob, opts = _tiny(n=16, N=7, T=0.7, kappa=0.1, flow=W.FLOW_ABC, fp=(1.0, 0.8, 0.6), prec=prec)
    opts = W.PararealOpts(**{**opts.__dict__, "mode": W.MODE_COARSE_GRID})
    u0 = W.fourier_field(prob.n, 12, n_modes=6, kmax=3.0)
    p = pr.problem_of(prob)
    p64 = pr.problem_of(W.Problem(n=16, kappa=0.1, flow=W.FLOW_ABC, fp=(1.0, 0.8, 0.6)))
    ref = gpu_serial(ctx, p64, opts, u0)
    prob64 = W.Problem(n=16, kappa=0.1, flow=W.FLOW_ABC, fp=(1.0, 0.8, 0.6))
    ores = parareal.solve(prob64, opts, u0, keep_history=True)
    tol = 1e-12 if prec == W.PREC_F64 else 1e-5
    for k in (1, 3):
        say(f"coarse-grid iterate k={k} prec={prec}")
        o = W.PararealOpts(**{**opts.__dict__, "max_iter": k})
        U, rep = pr.pr_parareal_solve(ctx, p, o, to_dev(u0), U_ref=ref)
        assert rep.iters == k and rep.m0 == 0
        Un = to_np(U)
        worst = max(rel_l2(Un[j + 1], h) for j, h in enumerate(ores.history[k]))
        say(f"  worst rel L2 vs oracle {worst:.3e}")
        assert worst <= tol
    if prec == W.PREC_F64:
        U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=ref)
        assert rep.iters == opts.N - 1 and rep.converged
        assert np.array_equal(to_np(U), to_np(ref))
    with pytest.raises(pr.PrError) as e:
        pr.pr_parareal_solve(ctx, pr.problem_of(W.Problem(n=6, kappa=0.1, flow=W.FLOW_ABC,
                                                          fp=(1.0, 1.0, 1.0))),
                             opts, to_dev(W.blob_field(6, 1)))
    assert e.value.name == "PR_EINVAL"


@pytest.mark.parametrize("mode", [W.MODE_ADAPTIVE, W.MODE_FIXED_POD], ids=["adaptive", "fixed"])
def test_coarse_gap_diagnostics_match_oracle(ctx, mode):
    """The coarse-gap diagnostics of Sec. 4 (dT = delta t: coarse_ratio 1)
    against the oracle's, step by step; the gaps are relative differences
    of iterates that agree to the round-off envelope, so they agree to
    about envelope / gap."""
    import paper_2601_10981_amd as pr
    prob, opts = _tiny(n=12, N=8, T=0.8, kappa=0.1, flow=W.FLOW_KOLMOGOROV, fp=(1.0, 2.0, 0.0))
    opts = W.PararealOpts(**{**opts.__dict__, "mode": mode, "diag": 1, "coarse_ratio": 1,
                             "max_iter": 3})
    u0 = W.fourier_field(prob.n, 9, n_modes=6, kmax=3.0)
    p = pr.problem_of(prob)
    ref = gpu_serial(ctx, p, opts, u0)
    oref = parareal.reference(prob, opts, u0)
    ores = parareal.solve(prob, opts, u0, U_ref=oref)
    U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=ref)
    assert rep.iters == 3
    for k in range(1, 4):
        say(f"gaps k={k} mode={mode}: gpu {rep.gap_fine.get(k)} oracle {ores.gap_fine[k]}")
        for name, g, o in (("fine", rep.gap_fine, ores.gap_fine), ("ref", rep.gap_ref, ores.gap_ref)):
            assert len(g[k]) == len(o[k]) == opts.N - 1 - k, (name, k)
            for a, b in zip(g[k], o[k]):
                assert abs(a - b) <= 1e-5 * b + 1e-9, (name, k, a, b)
    # without a reference only the fine-vs-coarse gap is recorded
    _, rep2 = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0))
    assert rep2.gap_ref == {} and rep2.gap_fine[1] == rep.gap_fine[1]


def test_coarse_gap_diagnostics_closed_form(ctx):
    """A single Fourier mode under a uniform flow: the gap is the time
    discretisation alone, |P4(dt lam)^n_f - P4(dT lam)^n_c| / |P4(dt lam)^n_f|."""
    import paper_2601_10981_amd as pr
    n, kappa, c = 10, 0.05, (0.6, -0.9, 0.4)
    prob = W.Problem(n=n, kappa=kappa, flow=W.FLOW_UNIFORM, fp=c)
    opts = W.PararealOpts(T=0.6, N=4, dt=0.01, cap0=4, cap=4, tol=0.0, coarse_ratio=5,
                          gamma1=1.0, gamma2=1.0, gamma3=1.0, mode=W.MODE_FIXED_POD, diag=1)
    h = 2 * math.pi / n
    x = np.arange(n) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    kv = (1, 2, -1)
    u0 = np.cos(kv[0] * X + kv[1] * Y + kv[2] * Z + 0.3)
    p = pr.problem_of(prob)
    ref = gpu_serial(ctx, p, opts, u0)
    U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=ref)
    assert rep.m0 == 2
    lam = (-kappa * sum(4.0 / h ** 2 * math.sin(k * h / 2) ** 2 for k in kv)
           - 1j * sum(cd * math.sin(k * h) / h for cd, k in zip(c, kv)))
    p4 = lambda z: 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    zF = p4(opts.T / opts.N / rep.n_f * lam) ** rep.n_f
    zG = p4(opts.T / opts.N / rep.n_c * lam) ** rep.n_c
    expect = abs(zF - zG) / abs(zF)
    say(f"closed-form gap {expect:.6e}; gpu {rep.gap_fine}")
    for k, row in rep.gap_fine.items():
        for g in row:
            assert abs(g - expect) <= 1e-6 * expect
    with pytest.raises(pr.PrError) as e:
        pr.pr_parareal_solve(ctx, p, W.PararealOpts(**{**opts.__dict__, "mode": W.MODE_COARSE_GRID}),
                             to_dev(u0))
    assert e.value.name == "PR_EINVAL"


def test_parareal_waves_and_streams_do_not_change_bits(ctx, monkeypatch):
    """The execution plan leaves every item's arithmetic alone. That covers:
    a memory budget that cuts the fine and sweep waves (wave slots reused
    within an iteration), the sweep cut into parts whose stage-2 POD runs on
    the second stream, no overlap at all, and the stage-1 POD run after the
    fine phase instead of per sweep part. Each gives the solve and its ranks
    bit for bit."""
    import paper_2601_10981_amd as pr
    say("parareal waves and streams bitwise")
    prob, opts = _tiny(n=16, N=14, T=1.4, max_iter=5)
    u0 = W.fourier_field(prob.n, 5, n_modes=6, kmax=2.5)
    p = pr.problem_of(prob)
    monkeypatch.setenv("PR_SWEEP_PARTS", "1")
    U1, rep1 = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0))
    monkeypatch.setenv("PR_SWEEP_PARTS", "3")
    U3, rep3 = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0))
    assert np.array_equal(to_np(U1), to_np(U3))
    assert rep1.ranks == rep3.ranks and rep1.jump == rep3.jump
    monkeypatch.setenv("PR_DEFER_POD1", "0")
    U0, rep0 = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0))
    monkeypatch.delenv("PR_DEFER_POD1")
    assert np.array_equal(to_np(U0), to_np(U3))
    assert rep0.ranks == rep3.ranks and rep0.jump == rep3.jump
    full = pr.pr_footprint(p, opts)
    ran = 0
    for frac in (0.8, 0.65, 0.5):
        with pr.Context(0, budget_bytes=int(frac * full)) as c:
            try:
                Ub, repb = pr.pr_parareal_solve(c, p, opts, to_dev(u0))
            except pr.PrError as e:
                assert e.name == "PR_ENOMEM"
                continue
            assert np.array_equal(to_np(Ub), to_np(U3)), frac
            assert repb.ranks == rep3.ranks and repb.jump == rep3.jump
            ran += 1
    assert ran >= 1
    monkeypatch.delenv("PR_SWEEP_PARTS")


@pytest.mark.parametrize("defer,small", [("0", "1"), ("1", "1"), ("1", "0")])
def test_parareal_stage1_cholqr_deferred_or_not(ctx, monkeypatch, defer, small):
    """The stage-1 modes M-orthonormalised by their own CholQR (defer 0) or
    left as W y / sqrt(lambda), their Cholesky factors applied to the
    diagonal blocks of the stage-2 Gram instead (defer 1). The stage-2 CholQR
    factor either comes from a Gram pass over the formed modes (small 0) or
    from C^T G C (small 1). Every combination gives the same iterates up to
    round-off and the oracle's stage-2 ranks, with p = 1 so W^k_n holds three
    stage-1 bases."""
    import paper_2601_10981_amd as pr
    say(f"parareal stage-1 CholQR deferred={defer} small={small}")
    prob, opts = _tiny(n=12, N=8, T=0.8, kappa=0.1, flow=W.FLOW_KOLMOGOROV, fp=(1.0, 2.0, 0.0))
    u0 = W.fourier_field(prob.n, 9, n_modes=6, kmax=3.0)
    p = pr.problem_of(prob)
    ores = parareal.solve(prob, opts, u0, keep_history=True)
    env = _roundoff_envelope(prob, opts, u0, ores, 3)
    monkeypatch.setenv("PR_DEFER_CHOLQR", defer)
    monkeypatch.setenv("PR_SMALL_CHOLQR", small)
    for k in (2, 3):
        o = W.PararealOpts(**{**opts.__dict__, "max_iter": k})
        U, rep = pr.pr_parareal_solve(ctx, p, o, to_dev(u0))
        assert rep.ranks[k - 1] == ores.ranks[k], (k, rep.ranks[k - 1], ores.ranks[k])
        Un = to_np(U)
        hist = ores.history[k]
        worst = max(rel_l2(Un[j + 1], hist[j]) for j in range(len(hist)))
        say(f"  k={k} worst iterate rel L2 vs oracle {worst:.3e} (round-off envelope {env[k]:.3e})")
        assert worst <= 10.0 * env[k] + 1e-12
    monkeypatch.delenv("PR_DEFER_CHOLQR")
    monkeypatch.delenv("PR_SMALL_CHOLQR")


def test_parareal_zero_initial_state(ctx):
    """u0 = 0: every snapshot and basis has rank 0, every state stays exactly
    zero and the first jump (0 / 0, taken as 0) ends the solve."""
    import paper_2601_10981_amd as pr
    say("parareal zero initial state")
    prob, opts = _tiny(tol=1e-8)
    p = pr.problem_of(prob)
    u0 = np.zeros(prob.n ** 3)
    U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0))
    assert rep.converged and rep.iters == 1 and rep.m0 == 0
    assert np.all(to_np(U) == 0.0)
    assert rep.jump == [0.0]


def test_nan_in_the_iterate_returns_enumeric(ctx):
    """A NaN in the state reaches the jump norms (formula4's correction
    carries it) and the solve stops with PR_ENUMERIC instead of reading it as
    a zero jump; the incremental (serving) path reports the same."""
    import torch
    import paper_2601_10981_amd as pr
    prob, opts = _tiny(n=12, N=6, T=0.6, max_iter=3)
    p = pr.problem_of(prob)
    u0 = W.blob_field(prob.n, 7)
    u0[5] = float("nan")
    say("NaN initial state: pr_parareal_solve")
    with pytest.raises(pr.PrError) as e:
        pr.pr_parareal_solve(ctx, p, opts, to_dev(u0))
    assert e.value.name == "PR_ENUMERIC"
    say("NaN initial state: pr_solve_begin / step / end")
    h = pr.pr_solve_begin(ctx, p, opts, to_dev(u0))
    for _ in range(opts.N):
        if pr.pr_solve_step_batch(ctx, [h])[0]:
            break
    assert pr.pr_solve_done(h)
    with pytest.raises(pr.PrError) as e:
        pr.pr_solve_end(ctx, h)
    assert e.value.name == "PR_ENUMERIC"
    torch.cuda.synchronize()


def test_nan_in_the_reference_shows_in_the_error_only(ctx):
    """A NaN in U_ref makes the reported error NaN (the error maximum keeps
    it) while the jumps, the iterate and the status are unaffected."""
    import paper_2601_10981_amd as pr
    prob, opts = _tiny(n=12, N=6, T=0.6, max_iter=2)
    p = pr.problem_of(prob)
    u0 = W.blob_field(prob.n, 7)
    ref = gpu_serial(ctx, p, opts, u0)
    U1, rep1 = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=ref)
    bad = ref.clone()
    bad[3, 17] = float("nan")
    U2, rep2 = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=bad)
    assert rep2.status == rep1.status
    assert rep2.jump == rep1.jump
    assert np.array_equal(to_np(U1), to_np(U2))
    assert all(math.isnan(e) for e in rep2.err)
    assert all(math.isfinite(e) for e in rep1.err)


@pytest.mark.parametrize("mode", [W.MODE_FIXED_POD, W.MODE_ADAPTIVE, W.MODE_COARSE_GRID],
                         ids=["fixed_pod", "adaptive", "coarse_grid"])
def test_warm_up_window_of_two_subintervals(ctx, mode):
    """T_0 = 2 DeltaT, the paper's Parareal-I window (Sec. 4): the window's
    states and the converged prefix bitwise equal the GPU serial solve, the
    iterates match the oracle (POD modes within its round-off envelope), and
    finite termination comes after N - 2 iterations."""
    import paper_2601_10981_amd as pr
    prob, opts = _tiny(n=12, N=8, T=0.8, kappa=0.1, flow=W.FLOW_KOLMOGOROV, fp=(1.0, 2.0, 0.0))
    opts = W.PararealOpts(**{**opts.__dict__, "mode": mode, "n_warm": 2})
    u0 = W.fourier_field(prob.n, 9, n_modes=6, kmax=3.0)
    p = pr.problem_of(prob)
    ref = gpu_serial(ctx, p, opts, u0)
    ores = parareal.solve(prob, opts, u0, keep_history=True)
    env = _roundoff_envelope(prob, opts, u0, ores, 2)
    for k in (1, 2):
        say(f"warm-up window 2 DeltaT, mode {mode}, iterate k={k}")
        o = W.PararealOpts(**{**opts.__dict__, "max_iter": k})
        U, rep = pr.pr_parareal_solve(ctx, p, o, to_dev(u0), U_ref=ref)
        assert rep.iters == k and rep.n_sub == opts.N - 2 and rep.m0 == ores.m0
        Un = to_np(U)
        for j in range(0, k + 3):
            assert np.array_equal(Un[j], to_np(ref[j])), (k, j)
        worst = max(rel_l2(Un[j + 2], h) for j, h in enumerate(ores.history[k]))
        say(f"  worst rel L2 vs oracle {worst:.3e} (envelope {env[k]:.3e})")
        assert worst <= 10.0 * env[k] + 1e-12
        if mode == W.MODE_ADAPTIVE:
            assert rep.ranks[k - 1] == ores.ranks[k]
        # the reported error of iterate k: U_n against the reference at its
        # own time (n + 2) DeltaT
        host = max(rel_l2(Un[j], to_np(ref[j])) for j in range(2, opts.N + 1))
        say(f"  reported error {rep.err[k]:.6e}, from the states {host:.6e}")
        assert abs(rep.err[k] - host) <= 1e-10 * host + 1e-15
    U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=ref)
    assert rep.iters == opts.N - 2 and rep.converged
    assert np.array_equal(to_np(U), to_np(ref))
    assert rep.err[-1] == 0.0


@pytest.mark.parametrize("prec,small_cholqr,bound", [
    (W.PREC_F64, "1", 1e-2), (W.PREC_F64, "0", 1e-12), (W.PREC_MIXED, "1", 1e-6)],
    ids=["f64", "f64_mode_gram", "mixed"])
def test_stage2_basis_m_orthonormal(ctx, monkeypatch, prec, small_cholqr, bound):
    """Loss of M-orthonormality, max_ij |(Psi^T M Psi - I)_ij|, of every
    stage-2 basis the sweep uses, read from the sweep's own Galerkin Gram
    (opts.diag). The case keeps every mode above the rank threshold tau_r
    (gamma = 1, caps above the ranks), so lambda_1 / lambda_m is as large as
    the rank rule allows. Bounds from the arithmetic:
    * FP64, CholQR factor from the coefficient Gram C^T G C (default): the
      rounding of the snapshot Gram G stays in the modes, about
      eps lambda_1 / lambda_m <= eps / tau_r = 2.2e-3 (1e-2 with margin);
    * FP64 with a Gram pass over the formed modes (PR_SMALL_CHOLQR=0): a few
      eps;
    * PR_MIXED (always the pass over the modes, in FP64, of modes stored in
      FP32): the FP32 rounding of the stored modes, a few units of 2^-24."""
    import paper_2601_10981_amd as pr
    monkeypatch.setenv("PR_SMALL_CHOLQR", small_cholqr)
    prob = W.Problem(n=12, kappa=0.05, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0), precision=prec)
    opts = W.PararealOpts(T=0.6, N=6, dt=0.01, cap0=12, cap=31, tol=0.0, max_iter=3,
                          gamma1=1.0, gamma2=1.0, gamma3=1.0, diag=1)
    u0 = W.fourier_field(prob.n, 21, n_modes=8, kmax=3.0)
    p = pr.problem_of(prob)
    _, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0))
    assert rep.iters == 3
    worst = 0.0
    for k in range(1, 4):
        row = rep.basis_orth[k]
        say(f"basis orthogonality k={k} {prec} small_cholqr={small_cholqr}: {row} "
            f"ranks {rep.ranks[k - 1]}")
        assert len(row) == opts.N - 1 - k
        for v in row:
            assert v == v and 0.0 <= v <= bound, (k, v)
            worst = max(worst, v)
    say(f"worst {worst:.3e} (bound {bound:.0e})")
