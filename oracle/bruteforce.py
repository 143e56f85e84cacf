"""Oracle pin (test infrastructure only): the minimiser for n <= 4 by support
enumeration, independent of coordinate descent and of the line search.

For every sign pattern sigma_ij in {-1, 0, +1} of the off-diagonal pairs the
l1 term is linear on the orthant it fixes, so the restricted problem
    min -log det A + tr(SA) + lam*(sum_i A_ii + 2*sum_{i<j} sigma_ij A_ij)
    subject to A_ij = 0 where sigma_ij = 0, A positive definite
is smooth and convex and is solved by damped Newton. The pattern whose
minimiser has the prescribed signs and satisfies |(S - A^{-1})_ij| <= lam on
its zero pairs meets the optimality condition 0 in dF(A) of Section 4,
eq. (subgradient1), and is the unique solution.
"""

from __future__ import annotations

import itertools

import numpy as np


def _restricted_newton(S, lam, sigma, pairs, max_iter=200):
    n = S.shape[0]
    basis = []
    for i in range(n):
        E = np.zeros((n, n))
        E[i, i] = 1.0
        basis.append(E)
    for (i, j), s in zip(pairs, sigma):
        if s != 0:
            E = np.zeros((n, n))
            E[i, j] = E[j, i] = 1.0
            basis.append(E)
    L = np.diag(np.ones(n))
    for (i, j), s in zip(pairs, sigma):
        L[i, j] = L[j, i] = s
    C = S + lam * L                      # linear term: tr(C A)

    def f(A):
        try:
            Lc = np.linalg.cholesky(A)
        except np.linalg.LinAlgError:
            return np.inf
        return -2.0 * np.sum(np.log(np.diag(Lc))) + np.sum(C * A)

    A = np.diag(1.0 / (np.diag(S) + lam))
    fa = f(A)
    for _ in range(max_iter):
        W = np.linalg.inv(A)
        g = np.array([np.sum((C - W) * E) for E in basis])
        H = np.array([[np.sum((W @ Et @ W) * Es) for Es in basis] for Et in basis])
        try:
            step = -np.linalg.solve(H, g)
        except np.linalg.LinAlgError:
            return None
        dec = -g @ step
        if dec < 1e-28:
            return A
        D = sum(s * E for s, E in zip(step, basis))
        t = 1.0
        while True:
            fn = f(A + t * D)
            if np.isfinite(fn) and fn <= fa - 0.25 * t * dec:
                break
            t *= 0.5
            if t < 1e-20:
                return A
        A = A + t * D
        fa = fn
        if np.max(np.abs(A)) > 1e12:
            return None                  # unbounded on this orthant
    return A


def solve(S: np.ndarray, lam: float, atol: float = 1e-9):
    """Unique minimiser for n <= 4 by enumeration; raises if none is found."""
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0]
    if n > 4:
        raise ValueError("enumeration is meant for n <= 4")
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    found = []
    for sigma in itertools.product((-1, 0, 1), repeat=len(pairs)):
        A = _restricted_newton(S, lam, sigma, pairs)
        if A is None:
            continue
        ok = True
        W = np.linalg.inv(A)
        G = S - W
        for (i, j), s in zip(pairs, sigma):
            if s == 0:
                if abs(G[i, j]) > lam + atol:
                    ok = False
                    break
            elif np.sign(A[i, j]) != s or abs(A[i, j]) < atol:
                ok = False
                break
        if ok:
            found.append((sigma, A))
    if len(found) != 1:
        raise RuntimeError(f"expected exactly one KKT pattern, found {len(found)}")
    return found[0][1]
