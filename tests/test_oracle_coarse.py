"""Pins of the oracle's coarse propagator (reduced Galerkin system, eq. 8 /
eq00 / eq13) and the augmentation (eqaug, eq12).

* L-invariant subspace: under a uniform velocity each pair {cos(k.x),
  sin(k.x)} is invariant under the FD operator, so the Galerkin system on a
  basis of such pairs is exact and the reduced RK4 with the fine step equals
  the fine RK4 to round-off.
* After augmentation the state lies in span(Psi), d is M-orthogonal to R and
  of unit M-norm; augmentation is skipped for a state already in span(R).
"""
import math

import numpy as np

import workloads as W
from oracle import coarse, fd, pod


def _grid(n):
    x = np.arange(n) * (2 * math.pi / n)
    return np.meshgrid(x, x, x, indexing="ij")


def _invariant_setup(n=10):
    op = fd.Operator(n, 0.05, fd.FLOW_UNIFORM, (0.6, -0.9, 0.4))
    X, Y, Z = _grid(n)
    ks = [(1, 0, 0), (1, 2, -1), (0, 3, 1)]
    cols = []
    for k in ks:
        a = k[0] * X + k[1] * Y + k[2] * Z
        cols += [np.cos(a).reshape(-1), np.sin(a).reshape(-1)]
    B = np.stack(cols, axis=1)
    h3 = op.h ** 3
    Psi, kept = pod.m_orthonormalise(B, h3)
    assert kept == 6
    u0 = (0.7 * np.cos(X + 0.3) + 0.2 * np.sin(X + 2 * Y - Z) - 0.5 * np.cos(3 * Y + Z + 1.0))
    return op, Psi, u0, h3


def test_invariant_subspace_coarse_equals_fine():
    op, Psi, u0, h3 = _invariant_setup()
    n_f, dt = 40, 0.01
    fine, _ = fd.fine_propagate(op, u0, dt, n_f)
    lifted, betas, nc = coarse.coarse_propagate(op, Psi, [u0.reshape(-1)], n_f * dt, n_f, h3)
    assert nc == n_f
    assert np.max(np.abs(lifted[0] - fine.reshape(-1))) <= 1e-13


def test_reduced_matrices_are_galerkin():
    op, Psi, u0, h3 = _invariant_setup()
    Lr, Mr = coarse.reduced_matrices(op, Psi, h3)
    assert np.max(np.abs(Mr - np.eye(6))) <= 1e-13
    # skew part from advection, negative-definite symmetric part from diffusion
    sym = 0.5 * (Lr + Lr.T)
    assert np.all(np.linalg.eigvalsh(sym) < 0)
    # Galerkin: L Psi = Psi K exactly in an invariant subspace
    K = np.linalg.solve(Mr, Lr)
    n = op.n
    for j in range(6):
        LP = op.apply(Psi[:, j].reshape(n, n, n)).reshape(-1)
        assert np.max(np.abs(LP - Psi @ K[:, j])) <= 1e-11 * max(1.0, np.max(np.abs(LP)))


def test_augmentation_contains_state():
    n = 8
    h3 = (2 * math.pi / n) ** 3
    Wm = W.random_matrix(n ** 3, 6, 21)
    R, m, _ = pod.pod_mode(Wm, 1.0, h3, cap=4)
    U = W.random_field(n, 22).reshape(-1)
    Psi, aug = coarse.augment(R, U, h3)
    assert aug and Psi.shape[1] == m + 1
    d = Psi[:, -1]
    assert abs(h3 * float(d @ d) - 1.0) <= 1e-13
    assert np.max(np.abs(h3 * (R.T @ d))) <= 1e-14
    Mr = h3 * (Psi.T @ Psi)
    Uproj = Psi @ np.linalg.solve(Mr, h3 * (Psi.T @ U))
    assert np.linalg.norm(Uproj - U) <= 1e-13 * np.linalg.norm(U)
    # state already in span(R): no augmentation
    U2 = R @ np.array([1.0, -2.0, 0.5, 0.25])
    Psi2, aug2 = coarse.augment(R, U2, h3)
    assert not aug2 and Psi2.shape[1] == m
    # empty basis: Psi = U / ||U||_M
    Psi3, aug3 = coarse.augment(np.zeros((n ** 3, 0)), U, h3)
    assert aug3 and np.allclose(Psi3[:, 0] * math.sqrt(h3 * float(U @ U)), U)


def test_stability_guard_doubles_steps():
    Lr = np.diag([-399.0, -1.0])
    Mr = np.eye(2)
    # ||K||_F = 399.00125: dT/n_c * ||K|| <= 2.5 needs n_c = 160 (10 doubled 4x)
    assert coarse.guarded_steps(Lr, Mr, 1.0, 10) == 160
    assert coarse.guarded_steps(Lr, Mr, 1.0, 200) == 200
    # a stable reduced RK4 keeps the decaying mode bounded
    b = coarse.reduced_rk4(Lr, Mr, np.array([1.0, 1.0]), 1.0, 160)
    assert abs(b[0]) < 1e-6 and abs(b[1] - math.exp(-1.0)) < 1e-8


def test_coarse_steps_reading():
    assert coarse.coarse_steps(63, 10) == 7
    assert coarse.coarse_steps(157, 10) == 16
    assert coarse.coarse_steps(5, 10) == 1
