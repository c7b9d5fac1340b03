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


def coarse_propagate(op, Psi: np.ndarray, states, dT_total: float, n_c: int, h3: float):
    """G(P U) for each U in ``states``: project onto span Psi, integrate the
    reduced system over dT_total, lift. Returns (lifted list, beta list, n_c
    after the guard)."""
    Lr, Mr = reduced_matrices(op, Psi, h3)
    n_c = guarded_steps(Lr, Mr, dT_total, n_c)
    lifted, betas = [], []
    for U in states:
        b = reduced_rk4(Lr, Mr, project(Psi, Mr, U, h3), dT_total, n_c)
        betas.append(b)
        lifted.append(Psi @ b if Psi.shape[1] else np.zeros(Psi.shape[0]))
    return lifted, betas, n_c
