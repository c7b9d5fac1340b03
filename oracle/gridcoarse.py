"""Coarse-grid coarse propagator of the oracle: the comparison method
"Parareal-II" of Sec. 4, whose coarse propagator discretises the same
equation on a coarser mesh (the paper: FEM with 8x fewer degrees of
freedom). Test infrastructure only, like the rest of the oracle.

On the finite-difference grid the coarse mesh is the n/2 node-centred grid
of the same periodic box (coarse node I sits on fine node 2I, 8x fewer
points), and the transfers are the standard pair:

  restriction (full weighting), per axis
      c[I] = 1/4 f[2I - 1] + 1/2 f[2I] + 1/4 f[2I + 1]
  prolongation (linear interpolation), per axis
      f[2I] = c[I],  f[2I + 1] = (c[I] + c[I + 1]) / 2

both periodic and applied axis by axis (so trilinear in 3-D). The coarse
propagator is G(u) = P(F_c(R u)) with F_c classical RK4 on the coarse grid
over DeltaT in n_g steps: n_g = max(1, ceil(n_f / coarse_ratio)) (the
paper's coarse step dT), doubled while dT * rho_c > 2.5 with rho_c =
12 kappa / h_c^2 + sum_d max|v_d| / h_c (max|v_d| from the flow's
coefficients), so the explicit coarse step stays inside RK4's stability
region.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import fd

GUARD = 2.5


def restrict(f: np.ndarray) -> np.ndarray:
    """Full weighting of an (n, n, n) field onto (n/2, n/2, n/2)."""
    c = np.asarray(f, dtype=np.float64)
    for axis in range(3):
        c = (0.25 * np.roll(c, 1, axis=axis) + 0.5 * c + 0.25 * np.roll(c, -1, axis=axis))
        c = np.take(c, np.arange(0, c.shape[axis], 2), axis=axis)
    return c


def prolong(c: np.ndarray) -> np.ndarray:
    """Linear interpolation of an (m, m, m) field onto (2m, 2m, 2m)."""
    f = np.asarray(c, dtype=np.float64)
    for axis in range(3):
        m = f.shape[axis]
        shape = list(f.shape)
        shape[axis] = 2 * m
        out = np.empty(shape)
        even = [slice(None)] * 3
        odd = [slice(None)] * 3
        even[axis] = slice(0, 2 * m, 2)
        odd[axis] = slice(1, 2 * m, 2)
        out[tuple(even)] = f
        out[tuple(odd)] = 0.5 * (f + np.roll(f, -1, axis=axis))
        f = out
    return f


def coarse_problem(prob):
    """The same problem on the n/2 grid."""
    if prob.n % 2 or prob.n // 2 < 4:
        raise ValueError("the coarse grid needs an even n with n/2 >= 4")
    return dataclasses.replace(prob, n=prob.n // 2)


def grid_steps(prob_c, dT: float, n_f: int, coarse_ratio: int) -> int:
    """Coarse RK4 steps over DeltaT: the coarse step rule, doubled while
    dT / n_g * rho_c > 2.5."""
    h = prob_c.L / prob_c.n
    rho = 12.0 * prob_c.kappa / (h * h) + fd.velocity_bound(prob_c.flow, prob_c.fp) / h
    n_g = max(1, int(math.ceil(n_f / float(coarse_ratio))))
    while dT / n_g * rho > GUARD:
        n_g *= 2
    return n_g


def coarse_grid_propagate(op_c, u: np.ndarray, dT: float, n_g: int, t0: float = 0.0) -> np.ndarray:
    """G(u) = P(F_c(R u)) for a fine field u (any shape with n^3 values), the
    coarse solve running over [t0, t0 + dT] (forced flows: with the forcing)."""
    m = op_c.n
    uc = restrict(np.asarray(u, dtype=np.float64).reshape(2 * m, 2 * m, 2 * m))
    vc, _ = fd.fine_propagate(op_c, uc, dT / n_g, n_g, t0=t0)
    return prolong(vc).reshape(-1)
