"""Oracle (test infrastructure only): the solution A*(lambda) by plain dense
proximal Newton on the full free set.

The estimator has a unique minimiser (Section 5, after eq. (MLE_l1_prior)),
so any correct solver defines the end-to-end result. This one is the plainest:
  1. W = A^{-1} by LAPACK Cholesky, G = S - W            (Section 5.1, eq. (gradHes))
  2. free set F = {A_ij != 0 or |G_ij| > lambda}          (Section 5.2, eq. (active_set))
  3. Newton direction: cyclic coordinate descent on the quadratic model
     restricted to F                                      (Section 5.1, eq. (Quad_MLE_l1_prior))
  4. step length: the backtracking rule of Section 6.1.2 with log det taken
     from a dense Cholesky of A + alpha*Delta (the plain definition that the
     block Schur-complement formula reaches)
  5. A <- A + alpha*Delta, repeat until the min-norm subgradient's max-norm
     is below ``tol``.
"""

from __future__ import annotations

import time

import numpy as np
import scipy.linalg as sla

from .cd import cd_sweeps
from .core import (covariance, free_mask, inverse_pd, kkt_l1, kkt_max,
                   logdet_identity_plus, objective)


def abs_change(a, d):
    """|a + d| - |a| elementwise without rounding a + d when no sign change occurs."""
    a = np.asarray(a, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    same = (a != 0) & (np.sign(a + d) == np.sign(a))
    return np.where(same, np.sign(a) * d, np.abs(a + d) - np.abs(a))


def objective_change(A, D, S, lam, L=None):
    """Return a function alpha -> F(A + alpha*D) - F(A) (inf when not PD).

    The change is formed term by term so that its rounding error scales with
    the step rather than with F itself:
        alpha*tr(S D) + lam*(||A + alpha D||_1 - ||A||_1)
        - [log det(A + alpha D) - log det A],
    with log det(A + alpha D) - log det A = log det(I + alpha L^{-1} D L^{-T})
    for A = L L^T, taken by ``core.logdet_identity_plus``.
    """
    if L is None:
        L = np.linalg.cholesky(A)
    Z = sla.solve_triangular(L, D, lower=True)
    Z = sla.solve_triangular(L, Z.T, lower=True)
    Z = 0.5 * (Z + Z.T)
    nzr, nzc = np.nonzero(D)
    trSD = float(np.sum(S[nzr, nzc] * D[nzr, nzc]))
    a0 = A[nzr, nzc]
    d0 = D[nzr, nzc]

    def dF(alpha):
        ld = logdet_identity_plus(alpha * Z)
        if ld is None:
            return float("inf")
        return alpha * trSD + lam * float(np.sum(abs_change(a0, alpha * d0))) - ld

    return dF


def linesearch_dense(A, D, S, lam, i_max: int = 30, beta: float = 0.5):
    """Step length for A + alpha*D (Section 6.1.2, Armijo variant).

    Reading: alpha = beta^i for i = 0, 1, ..., i_max; trials that are not
    positive definite are skipped; after the first PD trial the search goes on
    while the objective keeps decreasing and takes the best trial; if that
    trial does not decrease F (change >= 0), alpha = 0.
    Returns (alpha, F(A + alpha*D) - F(A), number of trials).
    """
    dF = objective_change(A, D, S, lam)
    best = None
    trials = 0
    for i in range(i_max + 1):
        a = beta ** i
        v = dF(a)
        trials += 1
        if not np.isfinite(v):
            continue
        if best is None or v < best[1]:
            best = (a, v)
            continue
        break
    if best is None or not best[1] < 0.0:
        return 0.0, 0.0, trials
    return best[0], best[1], trials


def solve(S: np.ndarray, lam: float, tol: float = 1e-10, max_iter: int = 200,
          A0: np.ndarray | None = None, verbose: bool = False, max_seconds: float | None = None):
    """Return (A*, info) with info['history'] = [(iter, F, kkt_max, nnz, seconds)].

    ``seconds`` is the time spent before the iteration's own work; with
    ``max_seconds`` the loop stops at the first iteration start past it.
    """
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0]
    A = np.eye(n) if A0 is None else np.array(A0, dtype=np.float64, copy=True)
    hist = []
    t0 = time.perf_counter()
    kkt = np.inf
    it = 0
    stalls = 0
    for it in range(max_iter):
        W = inverse_pd(A)
        G = S - W
        kkt = kkt_max(G, A, lam)
        F = objective(A, S, lam)
        hist.append((it, F, kkt, int(np.count_nonzero(A)), time.perf_counter() - t0))
        if verbose:
            print(f"[oracle] it={it} F={F:.15e} kkt={kkt:.3e} nnz={np.count_nonzero(A)}", flush=True)
        if kkt <= tol:
            break
        if max_seconds is not None and hist[-1][4] >= max_seconds:
            break
        mask = np.triu(free_mask(G, A, lam))
        ri, ci = np.nonzero(mask)
        inner_tol = max(1e-13, min(1e-3, kkt))
        D_vals, _, _ = cd_sweeps(W, ri, ci, S[ri, ci], A[ri, ci], lam,
                                 max_sweeps=200, tol=inner_tol, verbose=verbose)
        D = np.zeros_like(A)
        D[ri, ci] = D_vals
        D[ci, ri] = D_vals
        alpha, _, _ = linesearch_dense(A, D, S, lam)
        if alpha == 0.0:
            stalls += 1
            if stalls > 2:
                break
            continue
        A = A + alpha * D
    info = dict(history=hist, kkt_max=kkt, iterations=it,
                kkt_l1=kkt_l1(S - inverse_pd(A), A, lam),
                objective=objective(A, S, lam))
    return A, info


def solve_from_samples(X: np.ndarray, lam: float, **kw):
    return solve(covariance(X), lam, **kw)
