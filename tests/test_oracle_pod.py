"""Pins of the oracle's POD_Mode (Algorithm 1) against constructed spectra and
brute-force SVD.

* W = Q D V^T with M-orthonormal Q: the Gram W^T M W has eigenvalues d_i^2
  and eigenvectors V, so lambda, the rank and the modes are known by
  construction, and m follows from the sqrt(lambda) criterion by hand.
* For random W the M-orthogonal projector R R^T M of the kept modes equals
  the projector onto the leading left singular vectors of h^{3/2} W.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import pod


def _m_orthonormal(rows, cols, h3, seed):
    Q, _ = np.linalg.qr(W.random_matrix(rows, cols, seed))
    return Q / math.sqrt(h3)


def _orthogonal(k, seed):
    Q, _ = np.linalg.qr(W.random_matrix(k, k, seed))
    return Q


D = np.array([10.0, 3.0, 1.0, 0.3, 0.1, 0.01, 1e-4, 1e-9])


def _constructed(h3=(2 * math.pi / 8) ** 3):
    Q = _m_orthonormal(512, len(D), h3, 1)
    V = _orthogonal(len(D), 2)
    return Q, V, Q @ np.diag(D) @ V.T, h3


def test_constructed_spectrum_eigenvalues():
    Q, V, Wm, h3 = _constructed()
    lam, Y = pod.sorted_eigen(pod.gram(Wm, h3))
    # exact eigenvalues d^2; absolute error ~ eps * lambda_1
    assert np.max(np.abs(lam - D ** 2)) <= 1e-12 * D[0] ** 2
    # leading eigenvectors agree with V up to sign
    for j in range(5):
        assert abs(abs(float(Y[:, j] @ V[:, j])) - 1.0) <= 1e-12


def test_sqrt_lambda_criterion_by_hand():
    Q, V, Wm, h3 = _constructed()
    # sqrt(lambda) = d. r = #{d^2 > 1e-13 d_1^2} = 7 (1e-18 < 1e-11).
    # cumulative d: 10, 13, 14, 14.3, 14.4, 14.41, 14.4101; total 14.4101.
    # gamma = 0.99 -> 0.99 * 14.4101 = 14.266 -> m = 4.
    # (the same criterion on lambda instead of sqrt(lambda) would give m = 3)
    R, m, lam = pod.pod_mode(Wm, 0.99, h3, cap=10)
    assert m == 4
    R, m, lam = pod.pod_mode(Wm, 0.99, h3, cap=3)
    assert m == 3
    # gamma = 1: all r = 7 non-negligible modes
    R, m, lam = pod.pod_mode(Wm, 1.0, h3, cap=10)
    assert m == 7
    # gamma = 0.5: 10 >= 7.2 -> m = 1
    R, m, lam = pod.pod_mode(Wm, 0.5, h3, cap=10)
    assert m == 1


def test_constructed_modes_are_left_factors():
    Q, V, Wm, h3 = _constructed()
    R, m, lam = pod.pod_mode(Wm, 0.99, h3, cap=10)
    # r_i = W y_i / sqrt(lambda_i) = Q_i (up to sign)
    for j in range(m):
        c = h3 * float(R[:, j] @ Q[:, j])
        assert abs(abs(c) - 1.0) <= 1e-12


@pytest.mark.parametrize("rows,cols,seed", [(216, 6, 3), (343, 9, 4), (125, 12, 5)])
def test_projector_matches_brute_force_svd(rows, cols, seed):
    h3 = 0.37 ** 3
    Wm = W.random_matrix(rows, cols, seed) * np.logspace(0, -3, cols)
    R, m, lam = pod.pod_mode(Wm, 1.0, h3, cap=cols)
    assert m == cols
    U, s, _ = np.linalg.svd(math.sqrt(h3) * Wm, full_matrices=False)
    assert np.allclose(lam, s ** 2, rtol=1e-10, atol=1e-14 * s[0] ** 2)
    P_oracle = h3 * (R @ R.T)
    P_svd = U @ U.T
    assert np.max(np.abs(P_oracle - P_svd)) <= 1e-12
    # truncated: leading 3 modes
    R3, m3, _ = pod.pod_mode(Wm, 1.0, h3, cap=3)
    assert m3 == 3
    assert np.max(np.abs(h3 * (R3 @ R3.T) - U[:, :3] @ U[:, :3].T)) <= 1e-11


def test_modes_are_m_orthonormal():
    Wm = W.random_matrix(300, 10, 8) * np.logspace(0, -5, 10)
    h3 = 0.1
    R, m, _ = pod.pod_mode(Wm, 1.0, h3, cap=10)
    assert np.max(np.abs(h3 * (R.T @ R) - np.eye(m))) <= 1e-13


def test_zero_snapshots_give_empty_basis():
    R, m, lam = pod.pod_mode(np.zeros((64, 5)), 0.99, 1.0, cap=4)
    assert m == 0 and R.shape == (64, 0)


def test_force_m_and_rank_deficient_input():
    base = W.random_matrix(200, 3, 9)
    Wm = np.concatenate([base, base @ W.random_matrix(3, 4, 10)], axis=1)   # rank 3
    R, m, lam = pod.pod_mode(Wm, 1.0, 1.0, cap=7)
    assert m == 3
    assert np.all(lam[3:] <= 1e-13 * lam[0])
    R, m, _ = pod.pod_mode(Wm, 1.0, 1.0, cap=7, force_m=2)
    assert m == 2
    R, m, _ = pod.pod_mode(Wm, 1.0, 1.0, cap=7, force_m=6)
    assert m == 3


def test_eigenvector_sign_convention():
    G = np.array([[2.0, -1.0, 0.0], [-1.0, 2.0, -1.0], [0.0, -1.0, 2.0]])
    lam, Y = pod.sorted_eigen(G)
    assert np.all(np.diff(lam) <= 0)
    for j in range(3):
        i = int(np.argmax(np.abs(Y[:, j])))
        assert Y[i, j] > 0


def test_drop_pivot_rule_by_hand():
    """The re-orthonormalisation drops a mode whose M-norm squared residual
    against the earlier modes is <= 1e-8, together with every later one.
    Columns built from M-orthonormal vectors e_i with a known residual."""
    n3, h3 = 64, 0.1
    E = np.eye(n3)[:, :4] / math.sqrt(h3)         # M-orthonormal: h3 E^T E = I
    # third column: e_0 + eps e_2, residual M-norm^2 = eps^2
    for eps, kept in ((1e-5, 2), (1e-3, 4)):
        R = np.stack([E[:, 0], E[:, 1], E[:, 0] + eps * E[:, 2], E[:, 3]], axis=1)
        Q, m = pod.m_orthonormalise(R, h3)
        assert m == kept, (eps, m)
        assert Q.shape[1] == kept
        assert np.allclose(h3 * Q.T @ Q, np.eye(kept), atol=1e-12)
    # a repeated first column drops it and both later columns
    R = np.stack([E[:, 0], E[:, 0], E[:, 1]], axis=1)
    assert pod.m_orthonormalise(R, h3)[1] == 1
    # either side of the threshold: residual^2 below 1e-8 drops, above keeps
    for r2, kept in ((0.9e-8, 1), (1.1e-8, 2)):
        R = np.stack([E[:, 0], E[:, 0] + math.sqrt(r2) * E[:, 1]], axis=1)
        assert pod.m_orthonormalise(R, h3)[1] == kept, r2
