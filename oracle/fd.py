"""Fine propagator of the oracle: periodic FD operator and classical RK4.

The paper's fine propagator F (Sec. 2, formula1; Sec. 3.1) is P1 FEM with
implicit Euler. Here the spatial discretisation is second-order central finite
differences on a periodic node-centred n^3 grid and the time integrator is
classical RK4, applied to the semi-discrete system du/dt = L u with

    (L phi)_p = kappa * sum_d (phi_{p+e_d} - 2 phi_p + phi_{p-e_d}) / h^2
              - sum_d u_d(p) (phi_{p+e_d} - phi_{p-e_d}) / (2 h),

i.e. eq1 of Sec. 4 with c = 0, f = 0 and a steady divergence-free velocity.
Layout: arrays of shape (n, n, n) indexed [x][y][z] (z fastest).
"""
from __future__ import annotations

import math

import numpy as np

FLOW_UNIFORM = 0
FLOW_ABC = 1
FLOW_KOLMOGOROV = 2


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
    """The FD operator L of one problem (velocity sampled once)."""

    def __init__(self, n: int, kappa: float, flow: int, fp, L: float = 2 * math.pi):
        self.n = n
        self.kappa = float(kappa)
        self.h = spacing(n, L)
        self.vel = velocity(n, flow, fp, L)
        self.flow = flow
        self.fp = tuple(fp)

    @classmethod
    def of(cls, prob):
        return cls(prob.n, prob.kappa, prob.flow, prob.fp, prob.L)

    def apply(self, phi: np.ndarray) -> np.ndarray:
        """(L phi) with periodic wrap along every axis."""
        h = self.h
        lap = np.zeros_like(phi)
        adv = np.zeros_like(phi)
        for axis in range(3):
            plus = np.roll(phi, -1, axis=axis)    # phi_{p+e_d}
            minus = np.roll(phi, 1, axis=axis)    # phi_{p-e_d}
            lap += (plus - 2.0 * phi + minus) / (h * h)
            adv += self.vel[axis] * (plus - minus) / (2.0 * h)
        return self.kappa * lap - adv

    def spectral_bound(self) -> float:
        """Upper bound on |lambda(L)|: 12 kappa / h^2 + sum_d max|u_d| / h."""
        h = self.h
        return 12.0 * self.kappa / (h * h) + sum(float(np.max(np.abs(u))) for u in self.vel) / h


def rk4_step(op: Operator, phi: np.ndarray, dt: float) -> np.ndarray:
    """One classical RK4 step (k1..k4) of du/dt = L u."""
    k1 = op.apply(phi)
    k2 = op.apply(phi + 0.5 * dt * k1)
    k3 = op.apply(phi + 0.5 * dt * k2)
    k4 = op.apply(phi + dt * k3)
    return phi + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def velocity_bound(flow: int, fp) -> float:
    """sum_d max|v_d| from the flow's coefficients (not from grid samples):
    ABC (|A|+|C|) + (|B|+|A|) + (|C|+|B|), Kolmogorov |a|, uniform sum |c_d|."""
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
                   snap_every: int = 0):
    """F: n_steps RK4 steps from u0. With snap_every = dM > 0 it also returns
    the snapshot matrix W (N_g x n_s, one column per snapshot) holding the
    states at steps 0, dM, 2 dM, ... <= n_steps, so n_s = floor(n_steps/dM)+1
    (Sec. 3.2 Case I, the snapshot matrix W_h)."""
    phi = np.array(u0, dtype=np.float64, copy=True)
    snaps = []
    if snap_every > 0:
        snaps.append(phi.reshape(-1).copy())
    for j in range(1, n_steps + 1):
        phi = rk4_step(op, phi, dt)
        if snap_every > 0 and j % snap_every == 0:
            snaps.append(phi.reshape(-1).copy())
    if snap_every > 0:
        return phi, np.stack(snaps, axis=1)
    return phi, None


def serial_fine(op: Operator, u0: np.ndarray, dT_sub: float, N: int, dt_req: float):
    """Reference solution U_n of the error metric (eq. error): the fine
    propagator applied serially from the exact initial value, returned at
    t_n = n * DeltaT for n = 0..N (N + 1 fields)."""
    n_f, dt = steps_per_subinterval(dT_sub, dt_req)
    out = [np.array(u0, dtype=np.float64, copy=True)]
    phi = out[0]
    for _ in range(N):
        phi, _ = fine_propagate(op, phi, dt, n_f)
        out.append(phi)
    return out
