"""Pins of the oracle's fine propagator against closed forms.

* A single Fourier mode under a uniform velocity evolves by the FD symbol
  times the RK4 amplification polynomial: exact decay and translation.
* Under Kolmogorov shear an x-independent mode feels only diffusion.
* Every flow here has u_d independent of x_d, so the advection matrix is skew
  with A 1 = 0 and the Laplacian sums to zero: the field's sum is conserved.
* The ABC flow with A = B = C commutes with the cyclic permutation of axes.
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import fd


def _grid(n, L=2 * math.pi):
    x = np.arange(n) * (L / n)
    return np.meshgrid(x, x, x, indexing="ij")


def _p4(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def _symbol(k, c, kappa, h):
    lam = -(4 * kappa / h ** 2) * sum(math.sin(kd * h / 2) ** 2 for kd in k)
    lam = lam - 1j * sum(cd * math.sin(kd * h) / h for kd, cd in zip(k, c))
    return lam


@pytest.mark.parametrize("n,k,c,kappa", [
    (12, (1, 2, -3), (0.7, -0.4, 1.1), 0.03),
    (10, (4, 0, 1), (0.0, 2.0, -1.5), 0.2),
    (16, (-2, 5, 7), (1.3, 0.3, 0.0), 0.0),
])
def test_fourier_mode_uniform_flow(n, k, c, kappa):
    op = fd.Operator(n, kappa, fd.FLOW_UNIFORM, c)
    X, Y, Z = _grid(n)
    arg = k[0] * X + k[1] * Y + k[2] * Z
    phi0 = np.cos(arg)
    lam = _symbol(k, c, kappa, op.h)
    # one application of L: Re(lam e^{i k.x})
    Lphi = op.apply(phi0)
    exact_L = lam.real * np.cos(arg) - lam.imag * np.sin(arg)
    assert np.max(np.abs(Lphi - exact_L)) <= 1e-12 * max(1.0, abs(lam))
    dt = 0.3 / max(1.0, abs(lam))
    steps = 9
    phi, _ = fd.fine_propagate(op, phi0, dt, steps)
    R = _p4(dt * lam)
    exact = abs(R) ** steps * np.cos(arg + steps * np.angle(R))
    assert np.max(np.abs(phi - exact)) <= 1e-13


def test_kolmogorov_x_independent_mode_is_pure_diffusion():
    n, kappa = 16, 0.05
    op = fd.Operator(n, kappa, fd.FLOW_KOLMOGOROV, (1.3, 2.0, 0.0))
    X, Y, Z = _grid(n)
    phi0 = np.cos(2 * Y + 3 * Z)
    lam = -(4 * kappa / op.h ** 2) * (math.sin(2 * op.h / 2) ** 2 + math.sin(3 * op.h / 2) ** 2)
    dt, steps = 0.01, 25
    phi, _ = fd.fine_propagate(op, phi0, dt, steps)
    exact = _p4(dt * lam) ** steps * phi0
    assert np.max(np.abs(phi - exact)) <= 1e-13


def test_kolmogorov_advects_along_x():
    # u = (a sin(k_f y), 0, 0): a mode cos(x) at y with sin(k_f y) = 0 only
    # diffuses, and the advection term of L is -u_x d/dx exactly.
    n, a, kf = 16, 0.8, 2.0
    op = fd.Operator(n, 0.0, fd.FLOW_KOLMOGOROV, (a, kf, 0.0))
    X, Y, Z = _grid(n)
    phi0 = np.cos(X)
    Lphi = op.apply(phi0)
    exact = a * np.sin(kf * Y) * np.sin(X) * math.sin(op.h) / op.h
    assert np.max(np.abs(Lphi - exact)) <= 1e-13


@pytest.mark.parametrize("flow,fp", [(fd.FLOW_ABC, (1.0, 1.0, 1.0)),
                                     (fd.FLOW_ABC, (0.5, 1.5, 0.8)),
                                     (fd.FLOW_KOLMOGOROV, (1.0, 3.0, 0.0))])
def test_sum_conservation(flow, fp):
    n = 14
    op = fd.Operator(n, 0.04, flow, fp)
    phi0 = W.random_field(n, 11)
    phi, _ = fd.fine_propagate(op, phi0, 0.01, 30)
    s0, s1 = float(np.sum(phi0)), float(np.sum(phi))
    assert abs(s1 - s0) <= 1e-12 * float(np.sum(np.abs(phi0)))
    # and the flow really moves the field
    assert np.max(np.abs(phi - phi0)) > 1e-2


def test_abc_cyclic_permutation():
    n = 12
    op = fd.Operator(n, 0.05, fd.FLOW_ABC, (1.0, 1.0, 1.0))
    phi0 = W.random_field(n, 5)

    def perm(a):  # (P a)[i, j, k] = a[j, k, i]
        return np.transpose(a, (2, 0, 1))

    a, _ = fd.fine_propagate(op, perm(phi0), 0.02, 10)
    b, _ = fd.fine_propagate(op, phi0, 0.02, 10)
    assert np.max(np.abs(a - perm(b))) <= 1e-13
    # the permutation is not a symmetry of an asymmetric ABC flow
    op2 = fd.Operator(n, 0.05, fd.FLOW_ABC, (1.0, 0.5, 0.2))
    a2, _ = fd.fine_propagate(op2, perm(phi0), 0.02, 10)
    b2, _ = fd.fine_propagate(op2, phi0, 0.02, 10)
    assert np.max(np.abs(a2 - perm(b2))) > 1e-6


def test_step_count_reading():
    assert fd.steps_per_subinterval(1.0 / 8, 2e-3) == (63, 0.125 / 63)
    assert fd.steps_per_subinterval(10.0 / 64, 1e-3)[0] == 157
    assert fd.steps_per_subinterval(50.0 / 128, 5e-4)[0] == 782
    assert fd.steps_per_subinterval(5.0, 1e-2)[0] == 500   # the paper's 500 steps
    assert fd.snapshot_stride(63) == 4
    assert fd.snapshot_stride(157) == 10
    assert fd.snapshot_stride(782) == 49
    assert fd.snapshot_stride(500, 5) == 5


def test_automatic_step_rule():
    """dt <= 0 requests min(2e-3, 1.3 / rho) with rho = 12 kappa / h^2 +
    sum_d max|v_d| / h (values worked out by hand), and the step it gives
    is inside RK4's stability region for every discrete Fourier mode of a
    uniform flow (closed-form eigenvalues of L)."""
    P = W.Problem
    # n = 256, kappa = 0.1, ABC(1,1,1): rho = 1992.06 + 244.46 -> 5.8126e-4
    assert abs(fd.auto_dt(P(n=256, kappa=0.1, flow=fd.FLOW_ABC, fp=(1.0, 1.0, 1.0)))
               - 5.812608166e-4) <= 1e-12
    # n = 64, kappa = 0.01: rho = 73.57, 1.3 / rho > 2e-3 -> capped
    assert fd.auto_dt(P(n=64, kappa=0.01, flow=fd.FLOW_ABC, fp=(1.0, 1.0, 1.0))) == 2e-3
    # Kolmogorov counts only |a| (k_f does not enter): n = 128, kappa = 0.5,
    # a = -2: rho = 2490.07 + 40.74 -> 5.136689e-4
    a = fd.auto_dt(P(n=128, kappa=0.5, flow=fd.FLOW_KOLMOGOROV, fp=(-2.0, 1.0, 0.0)))
    b = fd.auto_dt(P(n=128, kappa=0.5, flow=fd.FLOW_KOLMOGOROV, fp=(-2.0, 4.0, 0.0)))
    assert a == b and abs(a - 5.136689e-4) <= 1e-10
    # stability: |P4(dt lambda(k))| <= 1 for every mode, uniform flow
    n, kappa, c = 16, 0.3, (3.0, -2.0, 1.5)
    prob = P(n=n, kappa=kappa, flow=fd.FLOW_UNIFORM, fp=c)
    dt = fd.auto_dt(prob)
    h = 2 * math.pi / n
    worst = 0.0
    for k in itertools.product(range(n), repeat=3):
        th = [2 * math.pi * kk / n for kk in k]
        lam = (-(4 * kappa / h ** 2) * sum(math.sin(t / 2) ** 2 for t in th)
               - 1j * sum(cd * math.sin(t) for cd, t in zip(c, th)) / h)
        z = dt * lam
        worst = max(worst, abs(1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24))
    assert worst <= 1.0


def test_snapshots_are_states_at_multiples_of_dM():
    n = 8
    op = fd.Operator(n, 0.1, fd.FLOW_ABC, (1.0, 1.0, 1.0))
    phi0 = W.random_field(n, 3)
    out, Wm = fd.fine_propagate(op, phi0, 0.01, 11, snap_every=4)
    assert Wm.shape == (n ** 3, 11 // 4 + 1)
    assert np.array_equal(Wm[:, 0], phi0.reshape(-1))
    p = phi0
    for j in range(1, 12):
        p = fd.rk4_step(op, p, 0.01)
        if j % 4 == 0:
            assert np.array_equal(Wm[:, j // 4], p.reshape(-1))
    assert np.array_equal(out, p)


def test_rk4_is_fourth_order_polynomial_of_L():
    # For linear autonomous L one RK4 step is P4(dt L) phi.
    n = 6
    op = fd.Operator(n, 0.07, fd.FLOW_ABC, (1.0, 0.6, 0.3))
    phi = W.random_field(n, 9)
    dt = 0.05
    terms = [phi]
    for j in range(1, 5):
        terms.append(op.apply(terms[-1]))
    poly = phi + dt * terms[1] + dt ** 2 / 2 * terms[2] + dt ** 3 / 6 * terms[3] + dt ** 4 / 24 * terms[4]
    assert np.max(np.abs(fd.rk4_step(op, phi, dt) - poly)) <= 1e-13


def _spectral_derivative(f, axis, L=2 * math.pi):
    """Exact derivative of a band-limited periodic field (FFT along axis)."""
    n = f.shape[axis]
    k = np.fft.fftfreq(n, d=L / n) * 2 * math.pi
    shape = [1, 1, 1]
    shape[axis] = n
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(f, axis=axis), axis=axis))


def test_abc_velocity_is_a_beltrami_field_with_its_amplitudes():
    """The ABC velocity (unequal A, B, C) is fixed without retyping it: it is
    divergence free, equals its own curl (a Beltrami field: curl u = u),
    each component's mean square is half the sum of the squares of its two
    amplitudes, and u(0, 0, 0) = (C, A, B). A sin <-> cos swap, a swapped
    amplitude or a sign slip in any component breaks one of these."""
    n, (A, B, C) = 16, (0.7, 1.3, 2.1)
    ux, uy, uz = fd.velocity(n, fd.FLOW_ABC, (A, B, C), 2 * math.pi)
    d = _spectral_derivative
    div = d(ux, 0) + d(uy, 1) + d(uz, 2)
    assert np.max(np.abs(div)) <= 1e-12
    curl = (d(uz, 1) - d(uy, 2), d(ux, 2) - d(uz, 0), d(uy, 0) - d(ux, 1))
    for c, u in zip(curl, (ux, uy, uz)):
        assert np.max(np.abs(c - u)) <= 1e-12
    for u, (a, b) in zip((ux, uy, uz), ((A, C), (B, A), (C, B))):
        assert abs(float(np.mean(u * u)) - 0.5 * (a * a + b * b)) <= 1e-12
    assert np.allclose([ux[0, 0, 0], uy[0, 0, 0], uz[0, 0, 0]], [C, A, B], rtol=0, atol=1e-15)


def test_kolmogorov_velocity_spectrum():
    """u = (a sin(k_f y), 0, 0): the x component depends on y alone, and its
    discrete Fourier transform along y is exactly -i a n / 2 at k_f and
    +i a n / 2 at -k_f (the transform of a sine), zero elsewhere."""
    n, a, kf = 16, 1.7, 3
    ux, uy, uz = fd.velocity(n, fd.FLOW_KOLMOGOROV, (a, float(kf), 0.0), 2 * math.pi)
    assert np.all(uy == 0.0) and np.all(uz == 0.0)
    assert np.all(ux == ux[:1, :, :1])          # a function of y only
    spec = np.fft.fft(ux[0, :, 0])
    expect = np.zeros(n, dtype=complex)
    expect[kf] = -0.5j * a * n
    expect[n - kf] = 0.5j * a * n
    assert np.max(np.abs(spec - expect)) <= 1e-12


@pytest.mark.parametrize("flow,fp", [(fd.FLOW_ABC, (0.7, 1.3, 2.1)),
                                     (fd.FLOW_KOLMOGOROV, (1.7, 3.0, 0.0))])
def test_steady_stencil_on_sinusoids_closed_form(flow, fp):
    """L on sin(x_d + c): the discrete Laplacian and central difference of a
    sinusoid are -(2 - 2 cos h) / h^2 and sin(h) / h times the sinusoid and
    its cosine, so L phi = kappa lap_f phi - u_d grad_f cos(x_d + c) with the
    velocity component u_d typed from the problem statement (unequal ABC
    amplitudes; Kolmogorov amplitude and wavenumber)."""
    n, kappa = 10, 0.3
    h = 2 * math.pi / n
    op = fd.Operator(n, kappa, flow, fp)
    X, Y, Z = _grid(n)
    if flow == fd.FLOW_ABC:
        A, B, C = fp
        U = (A * np.sin(Z) + C * np.cos(Y), B * np.sin(X) + A * np.cos(Z),
             C * np.sin(Y) + B * np.cos(X))
    else:
        a, kf = fp[0], fp[1]
        U = (a * np.sin(kf * Y), 0.0 * X, 0.0 * X)
    lap_f = -(2.0 - 2.0 * math.cos(h)) / h ** 2
    grad_f = math.sin(h) / h
    for d, (coord, c) in enumerate(((X, 0.3), (Y, -1.1), (Z, 2.0))):
        phi = np.sin(coord + c)
        expect = kappa * lap_f * phi - U[d] * grad_f * np.cos(coord + c)
        assert np.max(np.abs(op.apply(phi) - expect)) <= 1e-12
