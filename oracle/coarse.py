"""Coarse propagator of the oracle: POD-Galerkin reduced system (Sec. 3.2).

Given a basis Psi (N_g x q) of the POD subspace, the reduced system of eq. 8 /
eq00 uses the Galerkin matrices Psi^T A Psi and M_POD = Psi^T M Psi. With the
finite-difference operator L in place of the FEM stiffness, the semi-discrete
reduced system is

    M_r beta'(t) = L_r beta(t),   L_r = Psi^T M L Psi,  M_r = Psi^T M Psi,

and the Galerkin projection of a state U is beta = M_r^{-1} Psi^T M U.

Augmentation by the interface state (eqaug, eq12): d~ = U - R R^T M U,
d = d~ / ||d~||_M and Psi = [R, d]; eq13 is then the same Galerkin system over
the bordered basis (its lower-left blocks read d^T A R and d^T M R).

Readings where the paper is silent or differs from this discretisation:
  * Time integrator: the paper's coarse propagator uses the fine integrator
    with a coarse step; here that is classical RK4 in reduced coordinates with
    n_c = max(1, ceil(n_f / coarse_ratio)) steps over DeltaT.
  * Stability guard: while dT * ||M_r^{-1} L_r||_F > 2.5, n_c is doubled.
  * CGS2: the projection of eqaug is applied twice before normalising.
  * Degenerate augmentation (U in span R): skipped when
    ||d~||_M <= tau_aug ||U||_M, tau_aug = 1e-12.
  * M_r is kept explicitly (eq13 keeps Psi^T M Psi).
  * Forced, time-dependent flows (Sec. 4): the reduced system is
    M_r beta' = L_r(t) beta + f_r(t) with L_r(t) = Psi^T M L(t) Psi and
    f_r(t) = Psi^T M f(t), integrated by classical RK4 from the start time of
    the subinterval with stages at t, t + dT/2, t + dT/2, t + dT. The guard
    uses sum_j ||M_r^{-1} L_r,j||_F over the time-space pieces of the flow
    (fd.pieces: L(t) = L_0 + sum_{j>=1} theta_j(t) L_j with |theta_j| <= 1),
    which bounds ||M_r^{-1} L_r(t)||_F at every t and is the single Frobenius
    norm above for a steady flow.
"""
from __future__ import annotations

import math

import numpy as np

TAU_AUG = 1e-12
GUARD = 2.5


def reduced_matrices(op, Psi: np.ndarray, h3: float):
    """L_r = Psi^T M (L Psi), M_r = Psi^T M Psi for M = h^3 I."""
    n = op.n
    q = Psi.shape[1]
    LPsi = np.empty_like(Psi)
    for j in range(q):
        LPsi[:, j] = op.apply(Psi[:, j].reshape(n, n, n)).reshape(-1)
    Lr = h3 * (Psi.T @ LPsi)
    Mr = h3 * (Psi.T @ Psi)
    return Lr, Mr


def augment(R: np.ndarray, U: np.ndarray, h3: float, tau: float = TAU_AUG):
    """eqaug + eq12 (with CGS2). Returns (Psi, augmented?)."""
    u = U.reshape(-1)
    d = u - R @ (h3 * (R.T @ u))
    d = d - R @ (h3 * (R.T @ d))
    nd = math.sqrt(h3 * float(d @ d))
    nu = math.sqrt(h3 * float(u @ u))
    if nd > tau * nu and nd > 0.0:
        return np.concatenate([R, (d / nd)[:, None]], axis=1), True
    return R, False


def coarse_steps(n_f: int, coarse_ratio: int) -> int:
    return max(1, int(math.ceil(n_f / float(coarse_ratio))))


def guarded_steps(Lr: np.ndarray, Mr: np.ndarray, dT_total: float, n_c: int) -> int:
    """Double n_c until dT * ||M_r^{-1} L_r||_F <= 2.5."""
    if Lr.shape[0] == 0:
        return n_c
    K = np.linalg.solve(Mr, Lr)
    nrm = float(np.linalg.norm(K, "fro"))
    while (dT_total / n_c) * nrm > GUARD:
        n_c *= 2
    return n_c


def project(Psi: np.ndarray, Mr: np.ndarray, U: np.ndarray, h3: float) -> np.ndarray:
    """Galerkin projection coefficients beta = M_r^{-1} Psi^T M U."""
    if Psi.shape[1] == 0:
        return np.zeros(0)
    return np.linalg.solve(Mr, h3 * (Psi.T @ U.reshape(-1)))


def reduced_rk4(Lr: np.ndarray, Mr: np.ndarray, beta: np.ndarray,
                dT_total: float, n_c: int) -> np.ndarray:
    """n_c classical RK4 steps of M_r beta' = L_r beta over dT_total."""
    if beta.size == 0:
        return beta
    K = np.linalg.solve(Mr, Lr)
    dT = dT_total / n_c
    b = beta.copy()
    for _ in range(n_c):
        k1 = K @ b
        k2 = K @ (b + 0.5 * dT * k1)
        k3 = K @ (b + 0.5 * dT * k2)
        k4 = K @ (b + dT * k3)
        b = b + (dT / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return b


class ReducedSystem:
    """The Galerkin system of one basis Psi: M_r beta' = L_r beta for a steady
    flow, M_r beta' = L_r(t) beta + f_r(t) for a forced time-dependent one
    (L_r(t) and f_r(t) formed from their definitions at every stage time)."""

    def __init__(self, op, Psi: np.ndarray, h3: float):
        self.op = op
        self.Psi = Psi
        self.h3 = h3
        self.q = Psi.shape[1]
        self.forced = getattr(op, "forced", False)
        if self.forced:
            self.Mr = h3 * (Psi.T @ Psi)
            self.Lr = None
        else:
            self.Lr, self.Mr = reduced_matrices(op, Psi, h3)
        self._memo = {}

    def at(self, t: float):
        """K(t) = M_r^{-1} L_r(t) and g(t) = M_r^{-1} f_r(t)."""
        if t not in self._memo:
            n = self.op.n
            LPsi = np.empty_like(self.Psi)
            for j in range(self.q):
                LPsi[:, j] = self.op.apply(self.Psi[:, j].reshape(n, n, n), t).reshape(-1)
            Lr = self.h3 * (self.Psi.T @ LPsi)
            fr = self.h3 * (self.Psi.T @ self.op.forcing(t).reshape(-1))
            self._memo[t] = (np.linalg.solve(self.Mr, Lr), np.linalg.solve(self.Mr, fr))
        return self._memo[t]

    def piece_norm(self) -> float:
        """sum_j ||M_r^{-1} Psi^T M L_j Psi||_F over the flow's pieces."""
        from . import fd
        op = self.op
        n = op.n
        total = 0.0
        for j, (_, vel, _) in enumerate(fd.pieces(n, op.flow, op.fp, op.L)):
            LPsi = np.empty_like(self.Psi)
            for c in range(self.q):
                LPsi[:, c] = fd.apply_with(self.Psi[:, c].reshape(n, n, n), op.h,
                                           op.kappa if j == 0 else 0.0, vel).reshape(-1)
            K = np.linalg.solve(self.Mr, self.h3 * (self.Psi.T @ LPsi))
            total += float(np.linalg.norm(K, "fro"))
        return total

    def guarded_steps(self, dT_total: float, n_c: int) -> int:
        if not self.forced:
            return guarded_steps(self.Lr, self.Mr, dT_total, n_c)
        if self.q == 0:
            return n_c
        nrm = self.piece_norm()
        while (dT_total / n_c) * nrm > GUARD:
            n_c *= 2
        return n_c

    def rk4(self, beta: np.ndarray, t0: float, dT_total: float, n_c: int) -> np.ndarray:
        """n_c classical RK4 steps over [t0, t0 + dT_total]."""
        if not self.forced:
            return reduced_rk4(self.Lr, self.Mr, beta, dT_total, n_c)
        if beta.size == 0:
            return beta
        dT = dT_total / n_c
        b = beta.copy()
        for i in range(n_c):
            t = t0 + i * dT
            K1, g1 = self.at(t)
            K2, g2 = self.at(t + 0.5 * dT)
            k1 = K1 @ b + g1
            k2 = K2 @ (b + 0.5 * dT * k1) + g2
            k3 = K2 @ (b + 0.5 * dT * k2) + g2
            K4, g4 = self.at(t + dT)
            k4 = K4 @ (b + dT * k3) + g4
            b = b + (dT / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        return b

    def project(self, U: np.ndarray) -> np.ndarray:
        return project(self.Psi, self.Mr, U, self.h3)

    def lift(self, beta: np.ndarray) -> np.ndarray:
        return self.Psi @ beta if self.q else np.zeros(self.Psi.shape[0])


def coarse_propagate(op, Psi: np.ndarray, states, dT_total: float, n_c: int, h3: float,
                     t0: float = 0.0):
    """G(P U) for each U in ``states``: project onto span Psi, integrate the
    reduced system over [t0, t0 + dT_total], lift. Returns (lifted list, beta
    list, n_c after the guard)."""
    sysr = ReducedSystem(op, Psi, h3)
    n_c = sysr.guarded_steps(dT_total, n_c)
    lifted, betas = [], []
    for U in states:
        b = sysr.rk4(sysr.project(U), t0, dT_total, n_c)
        betas.append(b)
        lifted.append(Psi @ b if Psi.shape[1] else np.zeros(Psi.shape[0]))
    return lifted, betas, n_c
