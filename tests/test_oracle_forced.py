"""Pins of the oracle for the forced, time-dependent flows of Sec. 4 (the
Kolmogorov flow of eq. koleq and the ABC flow with phase sin(w t)).

* The time-space separation used for the reduced operators reproduces the
  flows as the paper writes them, at arbitrary times.
* The stencil on single sinusoids against the exact discrete derivatives
  (sin(h)/h and (2 - 2 cos h)/h^2 factors): pins the component-to-axis
  assignment, the sign of the advection, the time factor and the forcing.
* With kappa = 0 and no forcing, L(t) is skew-symmetric at every t (each
  velocity component is independent of its own coordinate).
* Pure forcing (a_v = 0, kappa = 0): one RK4 step is Simpson's rule, so the
  composite result matches the exact time integral within Simpson's bound;
  a wrong stage time breaks this at O(dt).
* Full problem: fourth-order convergence in dt against an independent
  adaptive integrator (scipy's DOP853) of the same semi-discrete system.
* A complete M-orthonormal basis makes the Galerkin reduced RK4 the full
  RK4 (pins the reduced forcing, stage times and the start time).
* The piece norm bounds ||M_r^{-1} L_r(t)||_F and equals it for a steady flow.
* Parareal finite termination with the forced flows (the subinterval start
  times line up with the serial reference).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import coarse, fd, parareal

FLOWS = [fd.FLOW_KOLMOGOROV_T, fd.FLOW_ABC_T]
L2PI = 2 * math.pi


def _grid(n):
    x = np.arange(n) * (L2PI / n)
    return np.meshgrid(x, x, x, indexing="ij")


@pytest.mark.parametrize("flow", FLOWS)
def test_separation_reproduces_the_flow(flow):
    n = 6
    fp = (0.7, -1.3, 1.9)
    parts = fd.pieces(n, flow, fp, L2PI)
    assert parts[0][0](123.0) == 1.0
    for t in (0.0, 0.37, 2.5, -4.1, 1005.0):
        (ux, uy, uz), f = fd.coefficients(n, flow, fp, L2PI, t)
        sv = [sum(th(t) * v[d] for th, v, _ in parts) for d in range(3)]
        sf = sum(th(t) * fj for th, _, fj in parts)
        for a, b in zip((ux, uy, uz), sv):
            assert np.allclose(a, b, rtol=0, atol=1e-14)
        assert np.allclose(f, sf, rtol=0, atol=1e-14)


def _paper_B_f(flow, X, Y, Z, t):
    # the flows of Sec. 4 at a_v = a_f = w = 1
    if flow == fd.FLOW_KOLMOGOROV_T:
        B = (np.cos(Y) + np.sin(Z) * np.cos(t), np.cos(Z) + np.sin(X) * np.cos(t),
             np.cos(X) + np.sin(Y) * np.cos(t))
        f = -np.cos(Y) - np.sin(Z) * np.cos(t)
    else:
        s = np.sin(t)
        B = (np.sin(Z + s) + np.cos(Y + s), np.sin(X + s) + np.cos(Z + s),
             np.sin(Y + s) + np.cos(X + s))
        f = -np.sin(Z + s) - np.cos(Y + s)
    return B, f


@pytest.mark.parametrize("flow", FLOWS)
def test_stencil_on_sinusoids_closed_form(flow):
    n, kappa, t = 10, 0.3, 0.81
    h = L2PI / n
    op = fd.Operator(n, kappa, flow, (1.0, 1.0, 1.0))
    X, Y, Z = _grid(n)
    B, f = _paper_B_f(flow, X, Y, Z, t)
    lap_f = -(2.0 - 2.0 * math.cos(h)) / h ** 2   # eigenvalue of the 1-D Laplacian
    grad_f = math.sin(h) / h                        # central difference of sin
    # one sinusoid per axis: phi = sin(x_d + c); D_d phi = grad_f cos(x_d + c)
    for d, (coord, c) in enumerate(((X, 0.3), (Y, -1.1), (Z, 2.0))):
        phi = np.sin(coord + c)
        expect = kappa * lap_f * phi - B[d] * grad_f * np.cos(coord + c)
        assert np.allclose(op.apply(phi, t), expect, rtol=0, atol=1e-12)
        assert np.allclose(op.rhs(phi, t), expect + f, rtol=0, atol=1e-12)


@pytest.mark.parametrize("flow", FLOWS)
def test_pure_advection_is_skew(flow):
    n = 8
    op = fd.Operator(n, 0.0, flow, (1.0, 0.0, 1.0))
    rng = np.random.default_rng(3)
    a = rng.standard_normal((n, n, n))
    b = rng.standard_normal((n, n, n))
    for t in (0.0, 0.9, 3.3):
        lhs = float(np.sum(a * op.apply(b, t)))
        rhs = -float(np.sum(op.apply(a, t) * b))
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1.0)
        assert abs(float(np.sum(a * op.apply(a, t)))) <= 1e-11 * float(np.sum(a * a))
    assert np.all(op.forcing(0.4) == 0.0)   # a_f = 0: no forcing


def test_pure_forcing_rk4_is_simpson():
    # u' = f(x, t) = a_f (-cos y - sin z cos(w t)): exact integral in closed form
    n, a_f, w = 6, 1.7, 2.3
    op = fd.Operator(n, 0.0, fd.FLOW_KOLMOGOROV_T, (0.0, a_f, w))
    X, Y, Z = _grid(n)
    u0 = np.cos(X) * 0.5
    t0, T, steps = 0.4, 1.2, 24
    dt = T / steps
    u, _ = fd.fine_propagate(op, u0, dt, steps, t0=t0)
    exact = u0 + a_f * (-np.cos(Y) * T - np.sin(Z) * (math.sin(w * (t0 + T)) - math.sin(w * t0)) / w)
    simpson = (T / 180.0) * dt ** 4 * a_f * w ** 4     # composite Simpson bound
    err = float(np.max(np.abs(u - exact)))
    assert err <= simpson
    # the same with the stage times shifted by dt/2 fails the bound by far
    assert float(np.max(np.abs(
        fd.fine_propagate(op, u0, dt, steps, t0=t0 + 0.5 * dt)[0] - exact))) > 100 * simpson


def test_pure_forcing_abc_against_quadrature():
    n, a_f, w = 4, 1.0, 1.0
    op = fd.Operator(n, 0.0, fd.FLOW_ABC_T, (0.0, a_f, w))
    u0 = np.zeros((n, n, n))
    t0, T, steps = 0.25, 1.0, 20
    u, _ = fd.fine_propagate(op, u0, T / steps, steps, t0=t0)
    x = np.arange(n) * (L2PI / n)
    for j in range(n):
        for k in range(n):
            g = lambda t: -math.sin(x[k] + math.sin(w * t)) - math.cos(x[j] + math.sin(w * t))
            ref, _ = integrate.quad(g, t0, t0 + T, epsabs=1e-12, epsrel=1e-12)
            assert abs(u[1, j, k] - ref) <= 1e-7
            assert np.allclose(u[:, j, k], u[0, j, k], atol=1e-15)   # no x dependence


@pytest.mark.parametrize("flow", FLOWS)
def test_rk4_fourth_order_against_dop853(flow):
    n, kappa = 6, 0.2
    op = fd.Operator(n, kappa, flow, (1.0, 1.0, 1.0))
    X, Y, Z = _grid(n)
    u0 = np.sin(X + 0.2) * np.cos(2 * Y) + 0.3 * np.cos(Z - Y)
    t0, T = 0.7, 0.6
    sol = integrate.solve_ivp(lambda t, y: op.rhs(y.reshape(n, n, n), t).reshape(-1),
                              (t0, t0 + T), u0.reshape(-1), method="DOP853",
                              rtol=1e-13, atol=1e-13)
    ref = sol.y[:, -1]
    errs = []
    for steps in (6, 12, 24):
        u, _ = fd.fine_propagate(op, u0, T / steps, steps, t0=t0)
        errs.append(float(np.max(np.abs(u.reshape(-1) - ref))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 12.0 < r2 < 20.0, errs


@pytest.mark.parametrize("flow", FLOWS)
def test_complete_basis_reduced_rk4_is_full_rk4(flow):
    n = 4
    op = fd.Operator(n, 0.1, flow, (1.0, 1.0, 1.0))
    h3 = op.h ** 3
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.standard_normal((n ** 3, n ** 3)))
    Psi = Q / math.sqrt(h3)                 # M-orthonormal, complete
    u0 = rng.standard_normal(n ** 3)
    t0, dT = 1.3, 0.2
    lifted, _, nc = coarse.coarse_propagate(op, Psi, [u0], dT, 3, h3, t0=t0)
    full, _ = fd.fine_propagate(op, u0.reshape(n, n, n), dT / nc, nc, t0=t0)
    assert np.allclose(lifted[0], full.reshape(-1), rtol=0, atol=1e-11 * np.max(np.abs(full)))
    # a different start time gives a different result (the time is used)
    other, _, _ = coarse.coarse_propagate(op, Psi, [u0], dT, 3, h3, t0=t0 + 0.5)
    assert np.max(np.abs(other[0] - lifted[0])) > 1e-4


@pytest.mark.parametrize("flow", FLOWS + [fd.FLOW_ABC])
def test_piece_norm_bounds_the_reduced_operator(flow):
    n = 6
    fp = (1.0, 1.0, 1.0)
    op = fd.Operator(n, 0.15, flow, fp)
    h3 = op.h ** 3
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((n ** 3, 7)))
    sysr = coarse.ReducedSystem(op, Q / math.sqrt(h3), h3)
    if flow == fd.FLOW_ABC:
        Lr, Mr = coarse.reduced_matrices(op, sysr.Psi, h3)
        K = np.linalg.solve(Mr, Lr)
        assert abs(sysr.piece_norm() - np.linalg.norm(K, "fro")) <= 1e-12 * np.linalg.norm(K)
        return
    bound = sysr.piece_norm()
    for t in np.linspace(0.0, 7.0, 15):
        K, _ = sysr.at(float(t))
        assert np.linalg.norm(K, "fro") <= bound * (1 + 1e-12)


@pytest.mark.parametrize("flow", FLOWS)
@pytest.mark.parametrize("mode", [W.MODE_ADAPTIVE, W.MODE_FIXED_POD, W.MODE_COARSE_GRID])
def test_forced_parareal_finite_termination(flow, mode):
    prob = W.Problem(n=8, kappa=0.1, flow=flow, fp=(1.0, 1.0, 1.0))
    opts = W.PararealOpts(T=0.5, N=5, dt=0.01, cap0=6, cap=8, tol=0.0, mode=mode)
    u0 = W.fourier_field(prob.n, 8, n_modes=6, kmax=3.0)
    ref = parareal.reference(prob, opts, u0)
    r = parareal.solve(prob, opts, u0, U_ref=ref, keep_history=True)
    assert r.iters == opts.N - 1
    for j in range(opts.N + 1):
        assert np.array_equal(r.U[j], ref[j].reshape(-1))
    for k, states in enumerate(r.history):
        for j in range(0, k + 1):
            assert np.array_equal(states[j], ref[j + 1].reshape(-1)), (k, j)


def test_forced_reference_differs_from_unforced():
    # the forcing drives a zero initial field away from zero
    prob = W.Problem(n=8, kappa=0.1, flow=fd.FLOW_KOLMOGOROV_T, fp=(1.0, 1.0, 1.0))
    opts = W.PararealOpts(T=0.4, N=4, dt=0.01)
    ref = parareal.reference(prob, opts, np.zeros((8, 8, 8)))
    assert np.max(np.abs(ref[-1])) > 0.1


@pytest.mark.parametrize("flow", FLOWS)
def test_grid_sum_conserved(flow):
    """Sum over the periodic grid is conserved: the Laplacian and the
    advection (each velocity component independent of its own coordinate)
    sum to zero, and so does the forcing (full periods of sin and cos)."""
    op = fd.Operator(16, 0.01, flow, (1.0, 1.0, 1.0))
    u = W.fourier_field(16, 3, n_modes=6, kmax=3.0) + 0.3
    v, _ = fd.fine_propagate(op, u, 0.01, 50, t0=7.0)
    assert abs(v.sum() - u.sum()) <= 1e-13 * np.abs(u).sum()
    assert np.max(np.abs(v - u)) > 1e-3      # the field did change
