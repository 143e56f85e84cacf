"""Oracle (test infrastructure only): objective, gradient, optimality measure.

Readings of the paper used throughout the oracle:
  * S = X^T X / m on X exactly as passed (no centring, no scaling); the
    estimator of Section 5 (eq. (cov_estimate)) centres the data, the workloads
    here draw zero-mean samples, so the plain second moment is used.
  * ||A||_1 sums |a_ij| over all entries, diagonal included, so an
    off-diagonal pair counts twice (Section 5, text after eq. (MLE_l1_prior)).
  * The free set uses a strict inequality |(S - A^{-1})_ij| > lambda and
    "A_ij != 0" means exactly non-zero (Section 5.2, eq. (active_set);
    Section 3, eq. (supp)).
  * The optimality measure is the min-norm subgradient of Section 4,
    eq. (subgradient1): m_ij = g_ij + lambda*sign(A_ij) on the support and
    sign(g_ij)*max(|g_ij| - lambda, 0) off it, with g = S - A^{-1}.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def covariance(X: np.ndarray) -> np.ndarray:
    """S = X^T X / m for the m x n sample matrix X (rows are samples)."""
    X = np.asarray(X, dtype=np.float64)
    return X.T @ X / X.shape[0]


def cholesky_lower(A: np.ndarray):
    """Lower Cholesky factor of a symmetric matrix, or None if not PD."""
    try:
        L = np.linalg.cholesky(np.asarray(A, dtype=np.float64))
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(L)):
        return None
    return L


def logdet_pd(A: np.ndarray):
    """log det A by Cholesky; None when A is not positive definite."""
    L = cholesky_lower(A)
    if L is None:
        return None
    return 2.0 * float(np.sum(np.log(np.diag(L))))


def logdet_identity_plus(E: np.ndarray, block: int = 128):
    """log det(I + E) for symmetric E, or None when I + E is not PD.

    Right-looking Cholesky of I + E with the identity kept implicit: the
    trailing-updated diagonal holds t_k with L_kk^2 = 1 + t_k, so
    log det(I + E) = sum_k log1p(t_k), which keeps full relative accuracy
    when E is small (forming 1 + t_k first would round t_k away).
    """
    E = np.array(E, dtype=np.float64, copy=True)
    n = E.shape[0]
    total = 0.0
    for k0 in range(0, n, block):
        k1 = min(k0 + block, n)
        for k in range(k0, k1):
            t = E[k, k]
            if not (1.0 + t > 0.0) or not np.isfinite(t):
                return None
            total += float(np.log1p(t))
            lkk = np.sqrt(1.0 + t)
            E[k + 1:k1, k] /= lkk
            col = E[k + 1:k1, k]
            E[k + 1:k1, k + 1:k1] -= np.outer(col, col)
        if k1 < n:
            # the loop left E[k, k] = t_k, so the pivots are sqrt(1 + t_k)
            d = np.sqrt(1.0 + np.diag(E[k0:k1, k0:k1]))
            L11 = np.tril(E[k0:k1, k0:k1], -1) + np.diag(d)
            L21 = sla.solve_triangular(L11, E[k1:, k0:k1].T, lower=True).T
            E[k1:, k1:] -= L21 @ L21.T
    return total


def inverse_pd(A: np.ndarray) -> np.ndarray:
    """A^{-1} for SPD A through its Cholesky factor (LAPACK potrf/potri)."""
    c, info = sla.lapack.dpotrf(np.asarray(A, dtype=np.float64), lower=0)
    if info != 0:
        raise np.linalg.LinAlgError("matrix is not positive definite")
    inv, info = sla.lapack.dpotri(c, lower=0)
    if info != 0:
        raise np.linalg.LinAlgError("potri failed")
    inv = np.triu(inv)
    return inv + np.triu(inv, 1).T


def objective(A: np.ndarray, S: np.ndarray, lam: float):
    """F(A) = -log det A + tr(SA) + lam * sum_ij |A_ij|  (Section 5, eq. (MLE_l1_prior)).

    Returns +inf when A is not positive definite.
    """
    ld = logdet_pd(A)
    if ld is None:
        return float("inf")
    return -ld + float(np.sum(S * A)) + lam * float(np.sum(np.abs(A)))


def gradient(A: np.ndarray, S: np.ndarray) -> np.ndarray:
    """grad f(A) = S - A^{-1}  (Section 5.1, eq. (gradHes))."""
    return S - inverse_pd(A)


def min_norm_subgradient(G: np.ndarray, A: np.ndarray, lam: float) -> np.ndarray:
    """Element of the subdifferential closest to 0 (Section 4, eq. (subgradient1))."""
    on = A != 0
    off_val = np.sign(G) * np.maximum(np.abs(G) - lam, 0.0)
    return np.where(on, G + lam * np.sign(A), off_val)


def kkt_max(G: np.ndarray, A: np.ndarray, lam: float) -> float:
    return float(np.max(np.abs(min_norm_subgradient(G, A, lam))))


def kkt_l1(G: np.ndarray, A: np.ndarray, lam: float) -> float:
    return float(np.sum(np.abs(min_norm_subgradient(G, A, lam))))


def free_mask(G: np.ndarray, A: np.ndarray, lam: float) -> np.ndarray:
    """Free set of Section 5.2, eq. (active_set): A_ij != 0 or |G_ij| > lam."""
    return (A != 0) | (np.abs(G) > lam)


def support_pairs(A: np.ndarray) -> np.ndarray:
    """Sorted keys i*n + j (i <= j) of the non-zeros of symmetric A."""
    n = A.shape[0]
    i, j = np.nonzero(np.triu(A != 0))
    return np.sort(i.astype(np.int64) * n + j)
