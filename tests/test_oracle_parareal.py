"""Pins of the oracle's adaptive parareal iteration (formula4, Algorithm 2).

* Finite termination (Sec. 2): after N' iterations the iterate equals the
  serial fine solution, and at every k the states U^k_j, j <= k, already do.
* L-invariant problem: when the snapshots span an L-invariant subspace and
  the coarse step equals the fine one, G = F and the k = 0 iterate is already
  the fine solution.
* The jumps of a converging run decrease and the final error is at the
  tolerance level.
* Fixed-POD mode ("Parareal-I" of Sec. 4): the same k = 0 step as the
  adaptive mode, finite termination, and one-iteration convergence when the
  k = 0 basis spans an L-invariant subspace (a wrong sign or a dropped term in
  the correction would leave the iterate off by a multiple of F).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fd, parareal


def _tiny(flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0), n=12, kappa=0.05, N=6, T=0.6,
          dt=0.01, tol=0.0, cap0=6, cap=8, ml=1, p=1, coarse_ratio=10, mode=W.MODE_ADAPTIVE):
    prob = W.Problem(n=n, kappa=kappa, flow=flow, fp=fp)
    opts = W.PararealOpts(T=T, N=N, dt=dt, cap0=cap0, cap=cap, tol=tol, ml=ml, p=p,
                          coarse_ratio=coarse_ratio, mode=mode)
    return prob, opts


@pytest.mark.parametrize("mode", [W.MODE_ADAPTIVE, W.MODE_FIXED_POD])
def test_finite_termination_and_prefix(mode):
    prob, opts = _tiny(mode=mode)
    u0 = W.blob_field(prob.n, 7)
    ref = parareal.reference(prob, opts, u0)
    r = parareal.solve(prob, opts, u0, U_ref=ref, keep_history=True)
    Np = opts.N - 1
    assert r.iters == Np
    for j in range(opts.N + 1):
        assert np.array_equal(r.U[j], ref[j].reshape(-1))
    # prefix property: U^k_j (parareal index j -> time index j + 1) exact for j <= k
    for k, states in enumerate(r.history):
        for j in range(0, k + 1):
            assert np.array_equal(states[j], ref[j + 1].reshape(-1)), (k, j)
    assert r.errors[-1] == 0.0


@pytest.mark.parametrize("ml,p", [(0, 0), (1, 0), (0, 1), (1, 1), (2, 1)])
def test_finite_termination_all_variants(ml, p):
    prob, opts = _tiny(N=5, T=0.5, ml=ml, p=p)
    u0 = W.fourier_field(prob.n, 8, n_modes=6, kmax=3.0)
    ref = parareal.reference(prob, opts, u0)
    r = parareal.solve(prob, opts, u0, U_ref=ref)
    assert r.iters == opts.N - 1
    assert r.errors[-1] == 0.0


def test_invariant_subspace_converges_at_k0():
    n = 10
    prob = W.Problem(n=n, kappa=0.05, flow=W.FLOW_UNIFORM, fp=(0.6, -0.9, 0.4))
    opts = W.PararealOpts(T=0.4, N=4, dt=0.01, cap0=8, cap=8, tol=1e-10,
                          coarse_ratio=1, gamma1=1.0, gamma2=1.0, gamma3=1.0)
    x = np.arange(n) * (2 * math.pi / n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    u0 = np.cos(X + 2 * Y - Z) + 0.5 * np.sin(3 * Y + Z + 0.4)
    ref = parareal.reference(prob, opts, u0)
    r = parareal.solve(prob, opts, u0, U_ref=ref)
    assert r.m0 == 4              # two cos/sin pairs
    assert r.errors[0] <= 1e-12   # G_0 = F on the invariant subspace
    assert r.iters == 1 and r.jumps[0] <= 1e-12


def test_converging_run_reaches_tolerance():
    prob, opts = _tiny(n=12, kappa=0.3, N=12, T=1.2, tol=1e-7, cap0=8, cap=12,
                       flow=W.FLOW_KOLMOGOROV, fp=(1.0, 2.0, 0.0))
    u0 = W.fourier_field(prob.n, 9, n_modes=6, kmax=3.0)
    ref = parareal.reference(prob, opts, u0)
    r = parareal.solve(prob, opts, u0, U_ref=ref)
    assert r.converged
    assert r.errors[-1] <= 1e-6
    assert all(b < a for a, b in zip(r.errors[:3], r.errors[1:4]))
    assert r.iters < opts.N - 1   # converged before finite termination
    assert r.jumps[-1] <= opts.tol


def test_zero_initial_field():
    prob, opts = _tiny(N=4, T=0.4)
    u0 = np.zeros((prob.n,) * 3)
    r = parareal.solve(prob, opts, u0)
    assert r.m0 == 0
    assert all(np.all(u == 0) for u in r.U)


def test_single_subinterval_is_plain_fine_solve():
    prob, opts = _tiny(N=1, T=0.1)
    u0 = W.random_field(prob.n, 4)
    ref = parareal.reference(prob, opts, u0)
    r = parareal.solve(prob, opts, u0)
    assert r.iters == 0 and len(r.U) == 2
    assert np.array_equal(r.U[1], ref[1].reshape(-1))


def test_fixed_pod_shares_the_k0_step_and_builds_no_bases():
    prob, opts = _tiny(N=5, T=0.5)
    fixed = W.PararealOpts(**{**opts.__dict__, "mode": W.MODE_FIXED_POD})
    u0 = W.fourier_field(prob.n, 8, n_modes=6, kmax=3.0)
    a = parareal.solve(prob, opts, u0, keep_history=True)
    b = parareal.solve(prob, fixed, u0, keep_history=True)
    assert a.m0 == b.m0
    for x, y in zip(a.history[0], b.history[0]):
        assert np.array_equal(x, y)
    assert all(len(v) == 0 for v in b.ranks.values())
    assert all(len(v) == 0 for v in b.ranks0.values())
    # the two coarse propagators differ after k = 0
    assert max(np.max(np.abs(x - y)) for x, y in zip(a.history[1], b.history[1])) > 1e-8


def test_fixed_pod_invariant_subspace_converges_in_one_iteration():
    n = 10
    prob = W.Problem(n=n, kappa=0.05, flow=W.FLOW_UNIFORM, fp=(0.6, -0.9, 0.4))
    opts = W.PararealOpts(T=0.4, N=4, dt=0.01, cap0=8, cap=8, tol=1e-10, coarse_ratio=1,
                          gamma1=1.0, gamma2=1.0, gamma3=1.0, mode=W.MODE_FIXED_POD)
    x = np.arange(n) * (2 * math.pi / n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    u0 = np.cos(X + 2 * Y - Z) + 0.5 * np.sin(3 * Y + Z + 0.4)
    ref = parareal.reference(prob, opts, u0)
    r = parareal.solve(prob, opts, u0, U_ref=ref)
    assert r.m0 == 4 and r.errors[0] <= 1e-12
    assert r.iters == 1 and r.jumps[0] <= 1e-12 and r.errors[1] <= 1e-12


@pytest.mark.parametrize("ratio", [1, 5])
def test_coarse_gap_diagnostics_closed_form(ratio):
    """Coarse-gap diagnostics (Sec. 4, dT = delta t runs) on a single Fourier
    mode under a uniform flow: span{cos, sin} is invariant under L, so the
    Galerkin reduction is exact in space and the gap is the time
    discretisation alone, |P4(dt lam)^n_f - P4(dT lam)^n_c| / |P4(dt lam)^n_f|
    with lam the FD symbol of the mode; it vanishes for dT = delta t. The
    reference gap at the first sweep step of iteration k starts from the
    exact U_k (converged prefix), so it takes the same value."""
    n, kappa, c = 10, 0.05, (0.6, -0.9, 0.4)
    prob = W.Problem(n=n, kappa=kappa, flow=W.FLOW_UNIFORM, fp=c)
    opts = W.PararealOpts(T=0.6, N=4, dt=0.01, cap0=4, cap=4, tol=0.0, coarse_ratio=ratio,
                          gamma1=1.0, gamma2=1.0, gamma3=1.0, mode=W.MODE_FIXED_POD, diag=1)
    h = 2 * math.pi / n
    x = np.arange(n) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    kv = (1, 2, -1)
    u0 = np.cos(kv[0] * X + kv[1] * Y + kv[2] * Z + 0.3)
    ref = parareal.reference(prob, opts, u0)
    r = parareal.solve(prob, opts, u0, U_ref=ref)
    assert r.m0 == 2
    lam = (-kappa * sum(4.0 / h ** 2 * math.sin(k * h / 2) ** 2 for k in kv)
           - 1j * sum(cd * math.sin(k * h) / h for cd, k in zip(c, kv)))
    p4 = lambda z: 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    dTs = opts.T / opts.N
    zF = p4(r.dt * lam) ** r.n_f
    zG = p4(dTs / r.n_c * lam) ** r.n_c
    expect = abs(zF - zG) / abs(zF)
    assert r.iters == opts.N - 1
    for k in range(1, r.iters + 1):
        assert len(r.gap_fine[k]) == opts.N - 1 - k
        for g in r.gap_fine[k]:
            assert abs(g - expect) <= 1e-9 * max(expect, 1e-6) + 1e-13
        if r.gap_ref[k]:
            assert abs(r.gap_ref[k][0] - expect) <= 1e-9 * max(expect, 1e-6) + 1e-13
    if ratio == 1:
        assert expect <= 1e-13
    else:
        assert expect > 1e-9


@pytest.mark.parametrize("ml,p", [(1, 1), (2, 1), (0, 1), (1, 0)])
def test_stage2_collection_is_the_papers_concatenation(ml, p):
    """W^k_n (Sec. 3.2 Case II, eq. W^k_n) is the column concatenation
    [R^k_{n-m_l,0}, ..., R^k_{n,0}, R^{k-1}_{n,0}, ..., R^{k-p}_{n,0}] of the
    stage-1 bases, built here by hand from the recorded bases with explicit
    indices. A block R^k_{j,0} that iteration k did not compute (j < k - 1:
    that subinterval had converged) is the latest one, from iteration j + 1;
    blocks with j < 0 or iteration < 1 are left out."""
    prob, opts = _tiny(N=7, T=0.7, ml=ml, p=p, cap0=4, cap=6)
    opts = W.PararealOpts(**{**opts.__dict__, "max_iter": 4})
    u0 = W.fourier_field(prob.n, 8, n_modes=6, kmax=3.0)
    tr = {}
    parareal.solve(prob, opts, u0, trace=tr)
    Np = opts.N - 1
    seen = 0
    for k in range(1, 5):
        for n in range(k, Np):
            R = lambda it, j: tr[("R0", it, j)]
            if (ml, p) == (1, 1):
                blocks = [R(k, n - 1), R(k, n)] + ([R(k - 1, n)] if k >= 2 else [])
            elif (ml, p) == (2, 1):
                blocks = []
                if n - 2 >= 0:
                    blocks.append(R(k - 1, n - 2) if n - 2 == k - 2 else R(k, n - 2))
                blocks += [R(k, n - 1), R(k, n)]
                blocks += [R(k - 1, n)] if k >= 2 else []
            elif (ml, p) == (0, 1):
                blocks = [R(k, n)] + ([R(k - 1, n)] if k >= 2 else [])
            else:
                blocks = [R(k, n - 1), R(k, n)]
            assert np.array_equal(tr[("W", k, n)], np.concatenate(blocks, axis=1)), (k, n)
            seen += 1
    assert seen == sum(Np - k for k in range(1, 5))
    # the n - 2 = k - 2 case of m_l = 2 takes the basis of iteration k - 1
    if ml == 2:
        assert ("R0", 3, 0) not in tr and ("R0", 2, 0) not in tr and ("R0", 1, 0) in tr


@pytest.mark.parametrize("mode", [W.MODE_FIXED_POD, W.MODE_ADAPTIVE, W.MODE_COARSE_GRID])
def test_warm_up_window_of_two_subintervals(mode):
    """T_0 = 2 DeltaT (the paper's Parareal-I set-up, Sec. 4): the window's
    states are the serial fine ones, the parareal partition of [T_0, T] has
    N - 2 subintervals and terminates after N - 2 iterations with the serial
    fine solution, and the k = 0 snapshots are the fine states at every dM
    steps across the whole window (checked against separate fine solves from
    u0 of j dM steps)."""
    prob, opts = _tiny(N=6, T=0.6, mode=mode, n=12)
    opts = W.PararealOpts(**{**opts.__dict__, "n_warm": 2, "dM": 3})
    u0 = W.fourier_field(prob.n, 8, n_modes=6, kmax=3.0)
    ref = parareal.reference(prob, opts, u0)
    r = parareal.solve(prob, opts, u0, U_ref=ref, keep_history=True)
    assert r.iters == opts.N - 2 and r.converged
    assert len(r.U) == opts.N + 1
    for j in range(opts.N + 1):
        assert np.array_equal(r.U[j], ref[j].reshape(-1)), j
    # the k = 0 iterate: U^0_0 is the fine state at T_0 = 2 DeltaT
    assert np.array_equal(r.history[0][0], ref[2].reshape(-1))
    assert len(r.history[0]) == opts.N - 1
    if mode == W.MODE_COARSE_GRID:
        return
    op = fd.Operator.of(prob)
    n_f, dt = fd.steps_per_subinterval(opts.T / opts.N, opts.dt)
    ends, Wh = fd.fine_window(op, u0, dt, n_f, 2, opts.dM)
    assert Wh.shape[1] == (2 * n_f) // opts.dM + 1
    for j in range(Wh.shape[1]):
        expect, _ = fd.fine_propagate(op, u0, dt, j * opts.dM)
        assert np.array_equal(Wh[:, j], expect.reshape(-1)), j
    assert np.array_equal(ends[0].reshape(-1), ref[1].reshape(-1))


def test_warm_up_window_one_is_the_default():
    prob, opts = _tiny(N=5, T=0.5)
    u0 = W.fourier_field(prob.n, 8, n_modes=6, kmax=3.0)
    a = parareal.solve(prob, opts, u0, keep_history=True)
    b = parareal.solve(prob, W.PararealOpts(**{**opts.__dict__, "n_warm": 1}), u0,
                       keep_history=True)
    assert a.iters == b.iters == opts.N - 1
    for x, y in zip(a.history[-1], b.history[-1]):
        assert np.array_equal(x, y)
