"""GPU parity of the forced, time-dependent flows of Sec. 4 (the Kolmogorov
flow of eq. koleq and the ABC flow with phase sin(w t)) against the oracle.

* fine propagator (classical RK4 with stage times and forcing): FP64
  relative L2 <= 1e-12 per field and snapshot, from several start times, on
  shapes with ragged tiles; FP32 stencil <= 1e-5; every tiling and x-chunk
  policy bitwise identical; a batch mixing steady and forced problems gives
  each item's solo result bitwise;
* coarse propagator (time-separable reduced operators, reduced forcing,
  augmentation, start time): <= 1e-11 and the same guarded step count;
* the parareal solve in all three modes: finite termination bitwise against
  the GPU serial solve, iterates against the oracle (POD modes within the
  oracle's own round-off envelope; the coarse-grid mode to 1e-12).
"""
import numpy as np
import pytest

import workloads as W
from oracle import coarse, fd, parareal, pod
from gpu_helpers import rel_l2, roundoff_envelope, say, to_dev, to_np

pytestmark = pytest.mark.gpu

KT, AT = W.FLOW_KOLMOGOROV_T, W.FLOW_ABC_T
PAPER = (1.0, 1.0, 1.0)

CASES = [
    # n, flow, fp, kappa, dt, steps, snap_every, t0, seed
    (20, KT, PAPER, 0.05, 0.01, 7, 2, 0.0, 1),
    (33, AT, PAPER, 0.1, 0.004, 5, 1, 2.7, 2),
    (40, KT, (0.7, 1.3, 2.0), 0.02, 0.008, 6, 3, 1003.5, 3),
    (24, AT, (1.2, -0.5, 0.5), 0.03, 0.01, 4, 4, 11.25, 4),
]


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_10981_amd as pr
    c = pr.Context(0)
    yield c
    c.close()


def _run(ctx, cases, prec=W.PREC_F64):
    import torch
    import paper_2601_10981_amd as pr
    items, outs, snaps = [], [], []
    fdt = torch.float32 if prec == W.PREC_MIXED else torch.float64
    for (n, flow, fp, kappa, dt, steps, se, t0, seed) in cases:
        uin = to_dev(W.random_field(n, seed))
        uout = torch.empty_like(uin)
        sn = torch.empty((steps // se + 1, n ** 3), dtype=fdt, device="cuda")
        items.append(dict(prob=pr.problem(n, kappa, flow, fp, prec), dt=dt, n_steps=steps,
                          u_in=uin, u_out=uout, snap_every=se, snaps=sn, t0=t0))
        outs.append(uout)
        snaps.append(sn)
    pr.pr_fine_propagate(ctx, items)
    torch.cuda.synchronize()
    return outs, snaps


def _oracle(case):
    n, flow, fp, kappa, dt, steps, se, t0, seed = case
    op = fd.Operator(n, kappa, flow, fp)
    out, Wm = fd.fine_propagate(op, W.random_field(n, seed), dt, steps, se, t0=t0)
    return out.reshape(-1), Wm


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}-flow{c[1]}-t{c[7]}")
def test_forced_fine_parity_f64(ctx, case):
    say(f"forced fine parity f64 {case}")
    outs, snaps = _run(ctx, [case])
    ref, Wm = _oracle(case)
    assert rel_l2(to_np(outs[0]), ref) <= 1e-12
    n = case[0]
    S = to_np(snaps[0]).reshape(-1, n ** 3)
    assert S.shape[0] == Wm.shape[1]
    for j in range(S.shape[0]):
        assert rel_l2(S[j], Wm[:, j]) <= 1e-12, j


@pytest.mark.parametrize("case", CASES[:2], ids=lambda c: f"n{c[0]}")
def test_forced_fine_mixed_precision(ctx, case):
    say(f"forced fine mixed {case}")
    outs, _ = _run(ctx, [case], W.PREC_MIXED)
    ref, _ = _oracle(case)
    assert rel_l2(to_np(outs[0]), ref) <= 1e-5


def test_forced_start_time_matters(ctx):
    # the same field from two start times differs (the time is read)
    a, _ = _run(ctx, [CASES[0]])
    b, _ = _run(ctx, [CASES[0][:7] + (0.9,) + CASES[0][8:]])
    assert rel_l2(to_np(a[0]), to_np(b[0])) > 1e-6


@pytest.mark.parametrize("prec", [W.PREC_F64, W.PREC_MIXED], ids=["f64", "mixed"])
def test_forced_every_tiling_is_bitwise_identical(ctx, prec, monkeypatch):
    say(f"forced tilings prec={prec}")
    ref_outs, ref_snaps = _run(ctx, CASES, prec)      # autotuned
    for pol in range(3):
        monkeypatch.setenv("PR_FUSED_CHUNK", str(pol))
        for cfg in range(5):
            monkeypatch.setenv("PR_FORCED_CFG", str(cfg))
            outs, snaps = _run(ctx, CASES, prec)
            for i in range(len(CASES)):
                assert np.array_equal(to_np(outs[i]), to_np(ref_outs[i])), (pol, cfg, i)
                assert np.array_equal(to_np(snaps[i]), to_np(ref_snaps[i])), (pol, cfg, i)
    monkeypatch.delenv("PR_FORCED_CFG")
    monkeypatch.delenv("PR_FUSED_CHUNK")


def test_forced_and_steady_in_one_batch(ctx):
    import torch
    import paper_2601_10981_amd as pr
    say("forced + steady batch")
    steady = (16, W.FLOW_ABC, (1.0, 1.0, 1.0), 0.05, 0.01, 6, 2, 0.0, 7)
    mix = [CASES[0], steady, CASES[1]]
    outs, snaps = _run(ctx, mix)
    for i, case in enumerate(mix):
        o1, s1 = _run(ctx, [case])
        assert np.array_equal(to_np(outs[i]), to_np(o1[0])), i
        assert np.array_equal(to_np(snaps[i]), to_np(s1[0])), i
    n, flow, fp, kappa, dt, steps, se, t0, seed = steady
    ref, _ = fd.fine_propagate(fd.Operator(n, kappa, flow, fp), W.random_field(n, seed), dt, steps)
    assert rel_l2(to_np(outs[1]), ref) <= 1e-12
    assert pr.pr_fine_tuned(ctx, pr.PR_F64, 20, 1, forced=True) is not None
    torch.cuda.synchronize()


def test_forced_stability_bound(ctx):
    import paper_2601_10981_amd as pr
    import torch
    # rho = 12 kappa / h^2 + 6 |a_v| / h; dt * rho > 2.6 is refused
    n = 16
    u = to_dev(W.random_field(n, 1))
    with pytest.raises(pr.PrError) as e:
        pr.pr_fine_propagate(ctx, [dict(prob=pr.problem(n, 0.0, KT, (1.0, 1.0, 1.0)), dt=0.2,
                                        n_steps=1, u_in=u, u_out=torch.empty_like(u))])
    assert e.value.name == "PR_EUNSTABLE"


def _coarse_setup_wide(n, flow, kappa, m, seed=3, t0=0.0):
    """An M-orthonormal basis of m smooth Fourier fields (any basis serves the
    coarse propagator) and states from a fine trajectory outside its span."""
    op = fd.Operator(n, kappa, flow, PAPER)
    h3 = op.h ** 3
    F = np.stack([W.fourier_field(n, seed + 11 * i, n_modes=4, kmax=2.5).reshape(-1)
                  for i in range(m)], axis=1)
    Q, _ = np.linalg.qr(F)
    R = Q / np.sqrt(h3)
    u0 = W.fourier_field(n, seed, n_modes=8, kmax=3.0)
    U1, _ = fd.fine_propagate(op, u0, 0.01, 40, t0=t0)
    U2 = U1 + 0.05 * W.random_field(n, seed + 7)
    return op, h3, R, U1.reshape(-1), U2.reshape(-1)


def _coarse_setup_smooth(n, flow, kappa, cap, seed=3, t0=0.0):
    op = fd.Operator(n, kappa, flow, PAPER)
    h3 = op.h ** 3
    u0 = W.fourier_field(n, seed, n_modes=8, kmax=3.0)
    _, Wm = fd.fine_propagate(op, u0, 0.01, 30, 2, t0=t0)
    R, m, _ = pod.pod_mode(Wm, 1 - 5e-6, h3, cap)
    U1, _ = fd.fine_propagate(op, u0, 0.01, 40, t0=t0)
    U2 = U1 + 0.05 * W.random_field(n, seed + 7)
    return op, h3, R, m, U1.reshape(-1), U2.reshape(-1)


@pytest.mark.parametrize("flow", [KT, AT], ids=["kolmogorov", "abc"])
@pytest.mark.parametrize("t0,dT,n_c", [(0.0, 0.2, 5), (3.4, 0.5, 2)])
def test_forced_coarse_parity(ctx, flow, t0, dT, n_c):
    import torch
    import paper_2601_10981_amd as pr
    say(f"forced coarse flow={flow} t0={t0}")
    n, cap, kappa = 12, 10, 0.05
    op, h3, R, m, U1, U2 = _coarse_setup_smooth(n, flow, kappa, cap, t0=t0)
    Psi, aug = coarse.augment(R, U1, h3)
    assert aug
    lifted, betas, nc = coarse.coarse_propagate(op, Psi, [U1, U2], dT, n_c, h3, t0=t0)
    Rp = np.zeros((n ** 3, cap))
    Rp[:, :m] = R
    ins = [to_dev(U1), to_dev(U2)]
    outs = [torch.empty_like(x) for x in ins]
    beta = torch.zeros((2, cap + 1), dtype=torch.float64, device="cuda")
    nco = torch.zeros(1, dtype=torch.int32, device="cuda")
    pr.pr_coarse_propagate(ctx, [dict(prob=pr.problem(n, kappa, flow, PAPER), R=to_dev(Rp.T),
                                      cap=cap, m=torch.tensor([m], dtype=torch.int32, device="cuda"),
                                      u_in=ins, dT_total=dT, n_c=n_c, u_out=outs, beta_out=beta,
                                      n_c_out=nco, u_aug=to_dev(U1), t0=t0)])
    torch.cuda.synchronize()
    assert int(nco.item()) == nc
    for o, l in zip(outs, lifted):
        assert rel_l2(to_np(o), l) <= 1e-11
    b = to_np(beta)
    for i in range(2):
        bg = np.concatenate([b[i, :m], b[i, cap:cap + 1]])
        assert np.max(np.abs(bg - betas[i])) <= 1e-11 * np.max(np.abs(betas[i]))


@pytest.mark.parametrize("flow", [KT, AT, W.FLOW_ABC], ids=["kolmogorov", "abc", "abc_steady"])
@pytest.mark.parametrize("cap", [20, 31])
def test_coarse_parity_wide_basis(ctx, flow, cap):
    """Bases of more than 16 columns: two MFMA tiles of basis columns, and
    the Galerkin blocks of every time-space piece packed up to nine tiles
    (31 columns, three pieces); the rank m = cap - 2 fills both tiles."""
    import torch
    import paper_2601_10981_amd as pr
    n, kappa, t0, dT, n_c = 12, 0.05, 1.3, 0.3, 3
    m = cap - 2
    op, h3, R, U1, U2 = _coarse_setup_wide(n, flow, kappa, m, t0=t0)
    say(f"forced coarse wide basis flow={flow} cap={cap} m={m}")
    Psi, aug = coarse.augment(R, U1, h3)
    lifted, betas, nc = coarse.coarse_propagate(op, Psi, [U1, U2], dT, n_c, h3, t0=t0)
    Rp = np.zeros((n ** 3, cap))
    Rp[:, :m] = R
    ins = [to_dev(U1), to_dev(U2)]
    outs = [torch.empty_like(x) for x in ins]
    beta = torch.zeros((2, cap + 1), dtype=torch.float64, device="cuda")
    nco = torch.zeros(1, dtype=torch.int32, device="cuda")
    pr.pr_coarse_propagate(ctx, [dict(prob=pr.problem(n, kappa, flow, PAPER), R=to_dev(Rp.T),
                                      cap=cap, m=torch.tensor([m], dtype=torch.int32, device="cuda"),
                                      u_in=ins, dT_total=dT, n_c=n_c, u_out=outs, beta_out=beta,
                                      n_c_out=nco, u_aug=to_dev(U1), t0=t0)])
    torch.cuda.synchronize()
    assert int(nco.item()) == nc
    # the basis is M-orthonormal to rounding, so the reduced solve is well
    # conditioned; the bound covers the Galerkin sums over 12^3 rows
    for o, l in zip(outs, lifted):
        assert rel_l2(to_np(o), l) <= 1e-10
    b = to_np(beta)
    for i in range(2):
        q = m + (1 if aug else 0)
        bg = np.concatenate([b[i, :m], b[i, cap:cap + 1]])[:q]
        assert np.max(np.abs(bg - betas[i])) <= 1e-10 * np.max(np.abs(betas[i]))


def gpu_serial(ctx, prob, opts, u0):
    """Serial fine solution on the GPU at t = j DeltaT; subinterval j starts
    at t = j DeltaT."""
    import torch
    import paper_2601_10981_amd as pr
    dTs = opts.T / opts.N
    n_f, dt = fd.steps_per_subinterval(dTs, opts.dt)
    out = torch.empty((opts.N + 1, prob.n ** 3), dtype=torch.float64, device="cuda")
    out[0].copy_(to_dev(u0))
    for j in range(opts.N):
        pr.pr_fine_propagate(ctx, [dict(prob=prob, dt=dt, n_steps=n_f, u_in=out[j], u_out=out[j + 1],
                                        t0=j * dTs)])
    torch.cuda.synchronize()
    return out


def _forced(flow, mode, n=12, N=8, T=0.8, kappa=0.1, prec=W.PREC_F64, **kw):
    prob = W.Problem(n=n, kappa=kappa, flow=flow, fp=PAPER, precision=prec)
    opts = W.PararealOpts(T=T, N=N, dt=0.01, cap0=6, cap=8, tol=0.0, mode=mode, **kw)
    return prob, opts


@pytest.mark.parametrize("flow", [KT, AT], ids=["kolmogorov", "abc"])
def test_forced_serial_matches_oracle(ctx, flow):
    import paper_2601_10981_amd as pr
    prob, opts = _forced(flow, W.MODE_ADAPTIVE, n=16, N=5, T=0.5)
    u0 = W.fourier_field(prob.n, 4, n_modes=6, kmax=3.0)
    ref = gpu_serial(ctx, pr.problem_of(prob), opts, u0)
    oref = parareal.reference(prob, opts, u0)
    for j in range(opts.N + 1):
        assert rel_l2(to_np(ref[j]), oref[j]) <= 1e-12, j


@pytest.mark.parametrize("flow", [KT, AT], ids=["kolmogorov", "abc"])
@pytest.mark.parametrize("mode", [W.MODE_ADAPTIVE, W.MODE_FIXED_POD, W.MODE_COARSE_GRID],
                         ids=["adaptive", "fixed", "grid"])
def test_forced_parareal_matches_oracle(ctx, flow, mode):
    import paper_2601_10981_amd as pr
    prob, opts = _forced(flow, mode)
    u0 = W.fourier_field(prob.n, 9, n_modes=6, kmax=3.0)
    p = pr.problem_of(prob)
    ref = gpu_serial(ctx, p, opts, u0)
    ores = parareal.solve(prob, opts, u0, keep_history=True)
    env = roundoff_envelope(prob, opts, u0, ores, 3) if mode != W.MODE_COARSE_GRID else [0.0] * 4
    for k in (1, 2, 3):
        say(f"forced parareal flow={flow} mode={mode} k={k}")
        o = W.PararealOpts(**{**opts.__dict__, "max_iter": k})
        U, rep = pr.pr_parareal_solve(ctx, p, o, to_dev(u0), U_ref=ref)
        assert rep.iters == k and rep.m0 == ores.m0
        Un = to_np(U)
        for j in range(0, k + 2):
            assert np.array_equal(Un[j], to_np(ref[j])), (k, j)
        if mode == W.MODE_ADAPTIVE:
            assert rep.ranks[k - 1] == ores.ranks[k], (k, rep.ranks[k - 1], ores.ranks[k])
        worst = max(rel_l2(Un[j + 1], h) for j, h in enumerate(ores.history[k]))
        say(f"  worst rel L2 vs oracle {worst:.3e} (envelope {env[k]:.3e})")
        assert worst <= 10.0 * env[k] + 1e-12
    U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=ref)
    assert rep.iters == opts.N - 1 and rep.converged
    assert np.array_equal(to_np(U), to_np(ref))


def test_forced_mixed_precision_converges(ctx):
    import paper_2601_10981_amd as pr
    prob, opts = _forced(KT, W.MODE_ADAPTIVE, n=16, N=8, T=0.8, prec=W.PREC_MIXED)
    opts = W.PararealOpts(**{**opts.__dict__, "tol": 1e-6, "cap0": 8, "cap": 12})
    u0 = W.fourier_field(prob.n, 5, n_modes=8, kmax=4.0)
    p64 = W.Problem(n=16, kappa=0.1, flow=KT, fp=PAPER)
    ref = gpu_serial(ctx, pr.problem_of(p64), opts, u0)
    U, rep = pr.pr_parareal_solve(ctx, pr.problem_of(prob), opts, to_dev(u0), U_ref=ref)
    say(f"forced mixed: iters {rep.iters} errs {rep.err}")
    assert rep.err[-1] <= 1e-5
    oref = parareal.reference(p64, opts, u0)
    assert rel_l2(to_np(U[-1]), oref[-1]) <= 1e-5


@pytest.mark.parametrize("mode", [W.MODE_ADAPTIVE, W.MODE_FIXED_POD], ids=["adaptive", "fixed"])
def test_forced_zero_initial_value(ctx, mode):
    """The paper's initial value h = 0 (Sec. 4): the warm-up snapshots start
    with a zero column, and the forcing alone drives the solution."""
    import paper_2601_10981_amd as pr
    prob, opts = _forced(KT, mode, n=12, N=6, T=0.6)
    u0 = np.zeros(prob.n ** 3)
    p = pr.problem_of(prob)
    ref = gpu_serial(ctx, p, opts, u0)
    ores = parareal.solve(prob, opts, u0, keep_history=True)
    o = W.PararealOpts(**{**opts.__dict__, "max_iter": 2})
    U, rep = pr.pr_parareal_solve(ctx, p, o, to_dev(u0), U_ref=ref)
    assert rep.iters == 2 and rep.m0 == ores.m0
    Un = to_np(U)
    env = roundoff_envelope(prob, opts, u0, ores, 2)
    worst = max(rel_l2(Un[j + 1], h) for j, h in enumerate(ores.history[2]))
    say(f"zero initial value mode={mode}: m0 {rep.m0}, worst rel L2 {worst:.3e} (envelope {env[2]:.3e})")
    assert worst <= 10.0 * env[2] + 1e-12
    U, rep = pr.pr_parareal_solve(ctx, p, opts, to_dev(u0), U_ref=ref)
    assert rep.iters == opts.N - 1 and np.array_equal(to_np(U), to_np(ref))
