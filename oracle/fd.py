"""Fine propagator of the oracle: periodic FD operator and classical RK4.

The paper's fine propagator F (Sec. 2, formula1; Sec. 3.1) is P1 FEM with
implicit Euler. Here the spatial discretisation is second-order central finite
differences on a periodic node-centred n^3 grid and the time integrator is
classical RK4, applied to the semi-discrete system du/dt = L u with

    (L phi)_p = kappa * sum_d (phi_{p+e_d} - 2 phi_p + phi_{p-e_d}) / h^2
              - sum_d u_d(p) (phi_{p+e_d} - phi_{p-e_d}) / (2 h),

i.e. eq1 of Sec. 4 with c = 0, f = 0 and a steady divergence-free velocity.

The two flows of Sec. 4 themselves (flows 3 and 4) have a time-dependent
velocity B(x, t) and a forcing f(x, t) (eq. koleq; the ABC flow with phase
sin(w t)); there the semi-discrete system is du/dt = L(t) u + f(t) with the
same stencil evaluated with B(., t), and one classical RK4 step from t takes
its stages at t, t + dt/2, t + dt/2, t + dt.
Layout: arrays of shape (n, n, n) indexed [x][y][z] (z fastest).
"""
from __future__ import annotations

import math

import numpy as np

FLOW_UNIFORM = 0
FLOW_ABC = 1
FLOW_KOLMOGOROV = 2
FLOW_KOLMOGOROV_T = 3   # the Kolmogorov flow of Sec. 4 (eq. koleq): B(t), f(t)
FLOW_ABC_T = 4          # the ABC flow of Sec. 4 with phase sin(w t): B(t), f(t)


def time_dependent(flow: int) -> bool:
    return flow in (FLOW_KOLMOGOROV_T, FLOW_ABC_T)


def _nodes(n: int, L: float):
    x = np.arange(n, dtype=np.float64) * spacing(n, L)
    return np.meshgrid(x, x, x, indexing="ij")


def coefficients(n: int, flow: int, fp, L: float, t: float):
    """B(x, t) = (u_x, u_y, u_z) and f(x, t) at the nodes for the forced flows
    of Sec. 4, written as the paper states them, with fp = (a_v, a_f, w)
    scaling the velocity and the forcing and setting the frequency (the
    paper's runs: a_v = a_f = w = 1):

      Kolmogorov (eq. koleq):
        B = a_v [(cos y, cos z, cos x) + (sin z, sin x, sin y) cos(w t)]
        f = a_f [-cos y - sin z cos(w t)]
      ABC with phase s = sin(w t):
        B = a_v (sin(z + s) + cos(y + s), sin(x + s) + cos(z + s),
                 sin(y + s) + cos(x + s))
        f = a_f [-sin(z + s) - cos(y + s)]
    """
    a_v, a_f, w = (float(v) for v in fp)
    X, Y, Z = _nodes(n, L)
    if flow == FLOW_KOLMOGOROV_T:
        c = math.cos(w * t)
        ux = a_v * (np.cos(Y) + np.sin(Z) * c)
        uy = a_v * (np.cos(Z) + np.sin(X) * c)
        uz = a_v * (np.cos(X) + np.sin(Y) * c)
        f = a_f * (-np.cos(Y) - np.sin(Z) * c)
    elif flow == FLOW_ABC_T:
        s = math.sin(w * t)
        ux = a_v * (np.sin(Z + s) + np.cos(Y + s))
        uy = a_v * (np.sin(X + s) + np.cos(Z + s))
        uz = a_v * (np.sin(Y + s) + np.cos(X + s))
        f = a_f * (-np.sin(Z + s) - np.cos(Y + s))
    else:
        raise ValueError(f"flow {flow} is not time-dependent")
    return (ux, uy, uz), f


def pieces(n: int, flow: int, fp, L: float):
    """The flows' separation in time and space (Sec. 4: B and f are separable):
    B(x, t) = sum_j theta_j(t) B_j(x), f(x, t) = sum_j theta_j(t) f_j(x),
    with theta_0 = 1. Returns [(theta_j, (u_x, u_y, u_z), f_j)]; steady flows
    have the single piece (1, v, 0).

      Kolmogorov: theta = (1, cos(w t)),
        B_0 = a_v (cos y, cos z, cos x),  f_0 = -a_f cos y,
        B_1 = a_v (sin z, sin x, sin y),  f_1 = -a_f sin z
      ABC with phase s = sin(w t): theta = (1, cos s, sin s),
        B_0 = 0, f_0 = 0,
        B_1 = a_v (sin z + cos y, sin x + cos z, sin y + cos x),
        f_1 = -a_f (sin z + cos y),
        B_2 = a_v (cos z - sin y, cos x - sin z, cos y - sin x),
        f_2 = -a_f (cos z - sin y)
    (sin(a + s) = sin a cos s + cos a sin s, cos(a + s) = cos a cos s -
    sin a sin s)."""
    if not time_dependent(flow):
        zero = np.zeros((n, n, n))
        return [(lambda t: 1.0, velocity(n, flow, fp, L), zero)]
    a_v, a_f, w = (float(v) for v in fp)
    X, Y, Z = _nodes(n, L)
    zero = np.zeros_like(X)
    if flow == FLOW_KOLMOGOROV_T:
        return [
            (lambda t: 1.0, (a_v * np.cos(Y), a_v * np.cos(Z), a_v * np.cos(X)), -a_f * np.cos(Y)),
            (lambda t: math.cos(w * t), (a_v * np.sin(Z), a_v * np.sin(X), a_v * np.sin(Y)),
             -a_f * np.sin(Z)),
        ]
    return [
        (lambda t: 1.0, (zero, zero, zero), zero),
        (lambda t: math.cos(math.sin(w * t)),
         (a_v * (np.sin(Z) + np.cos(Y)), a_v * (np.sin(X) + np.cos(Z)),
          a_v * (np.sin(Y) + np.cos(X))), -a_f * (np.sin(Z) + np.cos(Y))),
        (lambda t: math.sin(math.sin(w * t)),
         (a_v * (np.cos(Z) - np.sin(Y)), a_v * (np.cos(X) - np.sin(Z)),
          a_v * (np.cos(Y) - np.sin(X))), -a_f * (np.cos(Z) - np.sin(Y))),
    ]


def spacing(n: int, L: float) -> float:
    return L / n


def velocity(n: int, flow: int, fp, L: float):
    """Node values of the velocity (u_x, u_y, u_z), each an (n, n, n) array.

    ABC (A, B, C):  u = (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x)
    Kolmogorov (a, k_f): u = (a sin(k_f y), 0, 0)
    uniform (c_x, c_y, c_z): constant.
    """
    h = spacing(n, L)
    x = np.arange(n, dtype=np.float64) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    if flow == FLOW_ABC:
        A, B, C = fp
        ux = A * np.sin(Z) + C * np.cos(Y)
        uy = B * np.sin(X) + A * np.cos(Z)
        uz = C * np.sin(Y) + B * np.cos(X)
    elif flow == FLOW_KOLMOGOROV:
        a, kf = fp[0], fp[1]
        ux = a * np.sin(kf * Y)
        uy = np.zeros_like(X)
        uz = np.zeros_like(X)
    elif flow == FLOW_UNIFORM:
        ux = np.full_like(X, fp[0])
        uy = np.full_like(X, fp[1])
        uz = np.full_like(X, fp[2])
    else:
        raise ValueError(f"unknown flow {flow}")
    return ux, uy, uz


class Operator:
    """The FD operator L (or L(t)) of one problem. A steady velocity is
    sampled once; a time-dependent one (and its forcing) at each time asked
    for, from the paper's formulas (coefficients)."""

    def __init__(self, n: int, kappa: float, flow: int, fp, L: float = 2 * math.pi):
        self.n = n
        self.kappa = float(kappa)
        self.h = spacing(n, L)
        self.L = L
        self.flow = flow
        self.fp = tuple(fp)
        self.forced = time_dependent(flow)
        self.vel = None if self.forced else velocity(n, flow, fp, L)
        self._t = None
        self._coef = None

    @classmethod
    def of(cls, prob):
        return cls(prob.n, prob.kappa, prob.flow, prob.fp, prob.L)

    def _at(self, t: float):
        if self._t != t:
            self._coef = coefficients(self.n, self.flow, self.fp, self.L, t)
            self._t = t
        return self._coef

    def velocity_at(self, t: float = 0.0):
        return self._at(t)[0] if self.forced else self.vel

    def forcing(self, t: float = 0.0) -> np.ndarray:
        """f(., t) at the nodes (zero for the unforced flows)."""
        if not self.forced:
            return np.zeros((self.n, self.n, self.n))
        return self._at(t)[1]

    def apply(self, phi: np.ndarray, t: float = 0.0) -> np.ndarray:
        """(L(t) phi) with periodic wrap along every axis (no forcing)."""
        return apply_with(phi, self.h, self.kappa, self.velocity_at(t))

    def rhs(self, phi: np.ndarray, t: float = 0.0) -> np.ndarray:
        """L(t) phi + f(t): the right-hand side of the semi-discrete system."""
        r = self.apply(phi, t)
        if self.forced:
            r = r + self.forcing(t)
        return r

    def spectral_bound(self) -> float:
        """Upper bound on |lambda(L)|: 12 kappa / h^2 + sum_d max|u_d| / h."""
        h = self.h
        vel = self.velocity_at(0.0)
        return 12.0 * self.kappa / (h * h) + sum(float(np.max(np.abs(u))) for u in vel) / h


def apply_with(phi: np.ndarray, h: float, kappa: float, vel) -> np.ndarray:
    """kappa Lap_h phi - vel . grad_h phi (central differences, periodic)."""
    lap = np.zeros_like(phi)
    adv = np.zeros_like(phi)
    for axis in range(3):
        plus = np.roll(phi, -1, axis=axis)    # phi_{p+e_d}
        minus = np.roll(phi, 1, axis=axis)    # phi_{p-e_d}
        lap += (plus - 2.0 * phi + minus) / (h * h)
        adv += vel[axis] * (plus - minus) / (2.0 * h)
    return kappa * lap - adv


def rk4_step(op: Operator, phi: np.ndarray, dt: float, t: float = 0.0) -> np.ndarray:
    """One classical RK4 step (k1..k4) of du/dt = L(t) u + f(t) from time t:
    stages at t, t + dt/2, t + dt/2 and t + dt."""
    k1 = op.rhs(phi, t)
    k2 = op.rhs(phi + 0.5 * dt * k1, t + 0.5 * dt)
    k3 = op.rhs(phi + 0.5 * dt * k2, t + 0.5 * dt)
    k4 = op.rhs(phi + dt * k3, t + dt)
    return phi + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def velocity_bound(flow: int, fp) -> float:
    """sum_d max|v_d| from the flow's coefficients (not from grid samples):
    ABC (|A|+|C|) + (|B|+|A|) + (|C|+|B|), Kolmogorov |a|, uniform sum |c_d|;
    the two forced flows 6 |a_v| (each component is a sum of two terms of
    magnitude at most |a_v|, at every time)."""
    if time_dependent(flow):
        return 6.0 * abs(float(fp[0]))
    if flow == 1:
        A, B, C = (abs(float(v)) for v in fp)
        return (A + C) + (B + A) + (C + B)
    if flow == 2:
        return abs(float(fp[0]))
    return abs(float(fp[0])) + abs(float(fp[1])) + abs(float(fp[2]))


def auto_dt(prob) -> float:
    """Requested fine step when none is given: half of RK4's stability radius
    2.6 over rho = 12 kappa / h^2 + sum_d max|v_d| / h, at most 2e-3."""
    h = prob.L / prob.n
    rho = 12.0 * prob.kappa / (h * h) + velocity_bound(prob.flow, prob.fp) / h
    return min(2e-3, 0.5 * 2.6 / rho)


def steps_per_subinterval(dT_sub: float, dt_req: float):
    """Reading of the step count: n_f = ceil(DeltaT / dt_req - 1e-9) and the
    fine step delta_t = DeltaT / n_f, never larger than the requested step."""
    n_f = max(1, int(math.ceil(dT_sub / dt_req - 1e-9)))
    return n_f, dT_sub / n_f


def snapshot_stride(n_f: int, dM: int = 0) -> int:
    """delta_M (0 means ceil(n_f / 16), giving about 16 snapshots)."""
    return dM if dM > 0 else max(1, int(math.ceil(n_f / 16.0)))


def fine_propagate(op: Operator, u0: np.ndarray, dt: float, n_steps: int,
                   snap_every: int = 0, t0: float = 0.0):
    """F: n_steps RK4 steps from u0 at time t0 (step j starts at t0 + j dt).
    With snap_every = dM > 0 it also returns
    the snapshot matrix W (N_g x n_s, one column per snapshot) holding the
    states at steps 0, dM, 2 dM, ... <= n_steps, so n_s = floor(n_steps/dM)+1
    (Sec. 3.2 Case I, the snapshot matrix W_h)."""
    phi = np.array(u0, dtype=np.float64, copy=True)
    snaps = []
    if snap_every > 0:
        snaps.append(phi.reshape(-1).copy())
    for j in range(1, n_steps + 1):
        phi = rk4_step(op, phi, dt, t0 + (j - 1) * dt)
        if snap_every > 0 and j % snap_every == 0:
            snaps.append(phi.reshape(-1).copy())
    if snap_every > 0:
        return phi, np.stack(snaps, axis=1)
    return phi, None


def fine_window(op: Operator, u0: np.ndarray, dt: float, n_f: int, n_sub: int, dM: int):
    """The warm-up solve of Sec. 3.2 Case I over [0, T_0], T_0 = n_sub DeltaT
    (n_sub subintervals of n_f steps, from t = 0): the snapshot matrix W_h of
    the states at steps 0, dM, 2 dM, ... <= n_sub n_f (one contiguous
    sequence over the window, n_s = floor(n_sub n_f / dM) + 1 columns) and the
    states at the window's subinterval ends DeltaT, ..., n_sub DeltaT."""
    phi = np.array(u0, dtype=np.float64, copy=True)
    snaps = [phi.reshape(-1).copy()]
    ends = []
    for j in range(1, n_sub * n_f + 1):
        phi = rk4_step(op, phi, dt, (j - 1) * dt)
        if j % dM == 0:
            snaps.append(phi.reshape(-1).copy())
        if j % n_f == 0:
            ends.append(phi.copy())
    return ends, np.stack(snaps, axis=1)


def serial_fine(op: Operator, u0: np.ndarray, dT_sub: float, N: int, dt_req: float):
    """Reference solution U_n of the error metric (eq. error): the fine
    propagator applied serially from the exact initial value, returned at
    t_n = n * DeltaT for n = 0..N (N + 1 fields); subinterval i starts at
    t = i DeltaT."""
    n_f, dt = steps_per_subinterval(dT_sub, dt_req)
    out = [np.array(u0, dtype=np.float64, copy=True)]
    phi = out[0]
    for i in range(N):
        phi, _ = fine_propagate(op, phi, dt, n_f, t0=i * dT_sub)
        out.append(phi)
    return out
