"""Pins of the oracle's coarse-grid propagator ("Parareal-II", Sec. 4).

* The transfers: restriction and prolongation keep constants exactly; full
  weighting is the adjoint of linear interpolation up to the factor 8 (the
  ratio of cell volumes); prolongation reproduces the coarse values on the
  even fine nodes; restriction after prolongation multiplies a discrete
  Fourier mode of the coarse grid by prod_d (3/4 + cos(theta_d) / 4) (worked
  out by hand from the two stencils).
* The coarse step rule on hand-computed cases.
* The iteration: finite termination and the converged prefix, the k = 0 step
  shared with the other modes, and the k = 1 iterate composed by hand from
  F and G on three subintervals.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fd, gridcoarse as GC, parareal


def test_transfers_keep_constants_and_are_adjoint():
    f = np.full((8, 8, 8), 2.5)
    assert np.array_equal(GC.restrict(f), np.full((4, 4, 4), 2.5))
    assert np.array_equal(GC.prolong(np.full((4, 4, 4), -1.25)), np.full((8, 8, 8), -1.25))
    rng = np.random.Generator(np.random.PCG64(3))
    f = rng.standard_normal((12, 12, 12))
    c = rng.standard_normal((6, 6, 6))
    lhs = 8.0 * float(np.sum(GC.restrict(f) * c))
    rhs = float(np.sum(f * GC.prolong(c)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_prolongation_on_even_nodes_and_symbol_of_restrict_prolong():
    m = 6
    rng = np.random.Generator(np.random.PCG64(5))
    c = rng.standard_normal((m, m, m))
    assert np.array_equal(GC.prolong(c)[::2, ::2, ::2], c)
    I = np.arange(m)
    for k in [(1, 0, 0), (2, 1, 0), (1, 2, 3), (3, 3, 3)]:
        th = [2 * math.pi * kk / m for kk in k]
        mode = np.cos(th[0] * I[:, None, None] + th[1] * I[None, :, None] + th[2] * I[None, None, :])
        sym = np.prod([0.75 + 0.25 * math.cos(t) for t in th])
        assert np.max(np.abs(GC.restrict(GC.prolong(mode)) - sym * mode)) <= 1e-14


def test_grid_step_rule():
    # n = 16 -> coarse 8, h_c = pi/4; kappa 0.1, ABC(1,1,1): rho_c = 1.2/(pi/4)^2 + 6/(pi/4)
    # = 1.9454 + 7.6394 = 9.5848; dT = 0.5: ceil(50/10) = 5 steps, 0.1 * 9.58 = 0.96 <= 2.5
    pc = GC.coarse_problem(W.Problem(n=16, kappa=0.1, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0)))
    assert pc.n == 8
    assert GC.grid_steps(pc, 0.5, 50, 10) == 5
    # a step of 0.5 / 1 = 0.5: 4.79 > 2.5 -> 2 steps (2.40 <= 2.5)
    assert GC.grid_steps(pc, 0.5, 5, 10) == 2
    with pytest.raises(ValueError):
        GC.coarse_problem(W.Problem(n=13, kappa=0.1, flow=W.FLOW_ABC, fp=(1.0, 1.0, 1.0)))


def _setup(N=4, T=0.4, n=12):
    prob = W.Problem(n=n, kappa=0.1, flow=W.FLOW_KOLMOGOROV, fp=(1.0, 2.0, 0.0))
    opts = W.PararealOpts(T=T, N=N, dt=0.01, tol=0.0, mode=W.MODE_COARSE_GRID)
    u0 = W.fourier_field(n, 4, n_modes=6, kmax=3.0)
    return prob, opts, u0


def test_coarse_grid_finite_termination_and_prefix():
    prob, opts, u0 = _setup(N=6, T=0.6)
    ref = parareal.reference(prob, opts, u0)
    r = parareal.solve(prob, opts, u0, U_ref=ref, keep_history=True)
    assert r.iters == opts.N - 1 and r.errors[-1] == 0.0
    for j in range(opts.N + 1):
        assert np.array_equal(r.U[j], ref[j].reshape(-1))
    for k, states in enumerate(r.history):
        for j in range(k + 1):
            assert np.array_equal(states[j], ref[j + 1].reshape(-1)), (k, j)
    assert r.errors[0] > 1e-3          # the coarse grid is not exact


def test_coarse_grid_first_iterate_composed_by_hand():
    """N' = 3: U^1_1 = F(U^0_0), U^1_2 = G(U^1_1) + F(U^0_1) - G(U^0_1),
    U^1_3 = G(U^1_2) + F(U^0_2) - G(U^0_2), with U^0 the coarse sweep."""
    prob, opts, u0 = _setup(N=4, T=0.4)
    r = parareal.solve(prob, opts, u0, keep_history=True)
    op = fd.Operator.of(prob)
    pc = GC.coarse_problem(prob)
    opc = fd.Operator.of(pc)
    n_f, dt = fd.steps_per_subinterval(0.1, 0.01)
    n_g = GC.grid_steps(pc, 0.1, n_f, opts.coarse_ratio)
    F = lambda u: fd.fine_propagate(op, u.reshape((prob.n,) * 3), dt, n_f)[0].reshape(-1)
    G = lambda u: GC.coarse_grid_propagate(opc, u, 0.1, n_g)
    U0 = [F(u0)]
    for _ in range(3):
        U0.append(G(U0[-1]))
    for a, b in zip(U0, r.history[0]):
        assert np.max(np.abs(a - b)) <= 1e-14
    U1 = [U0[0], F(U0[0])]
    U1.append(G(U1[1]) + F(U0[1]) - G(U0[1]))
    U1.append(G(U1[2]) + F(U0[2]) - G(U0[2]))
    for a, b in zip(U1, r.history[1]):
        assert np.max(np.abs(a - b)) <= 1e-13
    # k = 0 starts from the same warm-up solve as the adaptive mode
    a = parareal.solve(prob, W.PararealOpts(**{**opts.__dict__, "mode": W.MODE_ADAPTIVE}), u0,
                       keep_history=True)
    assert np.array_equal(a.history[0][0], r.history[0][0])
