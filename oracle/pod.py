"""POD_Mode of the oracle (Algorithm 1; Sec. 3.2 Case I).

Given a snapshot matrix W (N_g x n_s) and the mass matrix M, POD_Mode solves
the eigenproblem of W^T M W, forms the modes r_i = W y_i / sqrt(lambda_i) and
keeps the first m of them, where m is the smallest k whose partial sum of
sqrt(lambda_i) reaches gamma times the sum over the r non-zero eigenvalues.

Readings where the paper is silent:
  * M = h^3 I for the finite-difference grid (the discrete L2 product).
  * "non-zero" eigenvalue: lambda_i > tau_r * lambda_1 (tau_r = 1e-13 for an
    FP64 Gram, 1e-6 for an FP32 Gram); no eigenvalue above that => m = 0.
  * m is capped at ``cap``; ``force_m`` (parity tests) replaces the criterion
    by min(force_m, r, cap).
  * Eigenvector sign: the entry of largest magnitude is positive (lowest
    index on ties).
  * The modes are re-orthonormalised in the M-inner product (QR of
    h^{3/2} R with a positive diagonal, i.e. the Gram-Schmidt order of the
    columns); a mode whose residual norm squared falls below 1e-8 is dropped
    together with all later ones.
"""
from __future__ import annotations

import numpy as np

TAU_R_F64 = 1e-13
TAU_R_F32 = 1e-6
DROP_PIVOT = 1e-8


def gram(W: np.ndarray, h3: float) -> np.ndarray:
    """G = W^T M W with M = h^3 I."""
    return h3 * (W.T @ W)


def sorted_eigen(G: np.ndarray):
    """Eigenpairs of the symmetric G, eigenvalues descending, eigenvectors
    sign-normalised (largest-magnitude entry positive, lowest index on ties)."""
    lam, Y = np.linalg.eigh(G)
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    Y = Y[:, order]
    for j in range(Y.shape[1]):
        i = int(np.argmax(np.abs(Y[:, j])))
        if Y[i, j] < 0:
            Y[:, j] = -Y[:, j]
    return lam, Y


def rank_from_spectrum(lam: np.ndarray, gamma: float, cap: int,
                       tau_r: float = TAU_R_F64, force_m=None) -> int:
    """Numerical rank r and the sqrt(lambda) criterion of Algorithm 1."""
    if lam.size == 0 or not (lam[0] > 0.0):
        return 0
    r = int(np.sum(lam > tau_r * lam[0]))
    if force_m is not None and force_m >= 0:
        return int(min(force_m, r, cap))
    s = np.sqrt(lam[:r])
    total = float(np.sum(s))
    acc = 0.0
    m = r
    for k in range(r):
        acc += float(s[k])
        if acc >= gamma * total:
            m = k + 1
            break
    return int(min(m, cap))


def m_orthonormalise(R: np.ndarray, h3: float):
    """Columns of R made M-orthonormal in their order (QR of h^{3/2} R with a
    positive diagonal). Returns (R', kept) where trailing columns from the
    first one with residual norm^2 <= DROP_PIVOT are dropped."""
    if R.shape[1] == 0:
        return R, 0
    s = np.sqrt(h3)
    Q, T = np.linalg.qr(s * R, mode="reduced")
    d = np.diag(T)
    sign = np.where(d < 0, -1.0, 1.0)
    Q = Q * sign
    piv = (d * d)
    kept = R.shape[1]
    for j in range(R.shape[1]):
        if piv[j] <= DROP_PIVOT:
            kept = j
            break
    return Q[:, :kept] / s, kept


def pod_mode(W: np.ndarray, gamma: float, h3: float, cap: int,
             tau_r: float = TAU_R_F64, force_m=None, reorth: int = 2):
    """Algorithm 1. Returns (R_tilde (N_g x m), m, lambda (descending)).

    ``reorth`` is the number of M-orthonormalisation passes applied to the
    modes (0 keeps the raw W y_i / sqrt(lambda_i) of the paper)."""
    G = gram(W, h3)
    lam, Y = sorted_eigen(G)
    m = rank_from_spectrum(lam, gamma, cap, tau_r, force_m)
    if m == 0:
        return np.zeros((W.shape[0], 0)), 0, lam
    R = W @ (Y[:, :m] / np.sqrt(lam[:m]))
    for _ in range(reorth):
        R, m = m_orthonormalise(R, h3)
    return R, m, lam
