"""Oracle (test infrastructure only): the block Newton direction by PCD-CG.

Section 6.1.1 solves the block subproblem (eq. (sub_Quad_MLE_l1_prior)) by
parallel coordinate descent accelerated by non-linear conjugate gradients; the
PCD step is the shrinkage step of Section 2 (eq. (IST_direction)) with D the
diagonal of the Hessian. The paper leaves the details to another reference,
so the steps below are this library's reading (stated with the GPU
implementation): Polak-Ribiere conjugation with restarts, and a line search
that takes the best of 64 step sizes on a geometric grid centred on the last
accepted step. Everything here is dense and plain: the Hessian product is
(W P W) formed with full matrices, the model is evaluated term by term.
"""

from __future__ import annotations

import numpy as np

GRID = 2.0 ** ((np.arange(64) - 32) / 8.0)   # candidate step sizes relative to the centre


def block_model(W, ri, ci, S_vals, A_vals, lam, D):
    """q(Delta) of eq. (sub_Quad_MLE_l1_prior) on the free coordinates (ri, ci)
    of W (local indices), with Delta symmetric: the linear and l1 terms count
    an off-diagonal pair twice, the quadratic term is 0.5 tr(W Delta W Delta)."""
    W = np.asarray(W, dtype=np.float64)
    nj = W.shape[0]
    M = np.zeros((nj, nj))
    M[ri, ci] = D
    M[ci, ri] = D
    gam = np.where(ri == ci, 1.0, 2.0)
    g = S_vals - W[ri, ci]
    return (np.sum(gam * (g * D + lam * np.abs(A_vals + D)))
            + 0.5 * np.trace(W @ M @ W @ M))


def l1_change(x, s):
    """|x + s| - |x| term by term; where x + s keeps the sign of x this is +-s
    exactly (near the minimiser the steps are far below |x|, and the difference
    of two sums of |x| would lose them to rounding)."""
    y = x + s
    keep_pos = (x > 0) & (y >= 0)
    keep_neg = (x < 0) & (y <= 0)
    return np.where(keep_pos, s, np.where(keep_neg, -s, np.abs(y) - np.abs(x)))


def hessian_product(W, ri, ci, p):
    """(W P W) at the free coordinates, P the symmetric matrix with entries p."""
    nj = W.shape[0]
    P = np.zeros((nj, nj))
    P[ri, ci] = p
    P[ci, ri] = p
    return (W @ P @ W)[ri, ci]


def pcd_cg(W, ri, ci, S_vals, A_vals, lam, max_iter=200, tol=1e-4, snap=True):
    """Returns (Delta per coordinate, iterations, max |alpha p| of the last step).

    One iteration: the PCD direction d (every coordinate's own 1-D minimiser
    at the current Delta, eq. (1d_l1) in parallel), p = d + beta p_prev, the
    exact model along p on the step-size grid, Delta += alpha p. Stops when
    max |alpha p| <= tol max |Delta|, when a restart gives no decrease, or after
    max_iter line searches. Finally (snap) every coordinate whose own 1-D
    minimiser is zero (x_k + d_k = 0) is set to exactly zero.
    """
    W = np.asarray(W, dtype=np.float64)
    ri = np.asarray(ri, dtype=np.int64)
    ci = np.asarray(ci, dtype=np.int64)
    S_vals = np.asarray(S_vals, dtype=np.float64)
    A_vals = np.asarray(A_vals, dtype=np.float64)
    nc = ri.size
    gam = np.where(ri == ci, 1.0, 2.0)
    g = S_vals - W[ri, ci]
    a = np.where(ri == ci, W[ci, ci] ** 2, W[ri, ci] ** 2 + W[ri, ri] * W[ci, ci])
    D = np.zeros(nc)
    z = np.zeros(nc)                 # W Delta W at the coordinates
    p_prev = np.zeros(nc)
    d_prev = np.zeros(nc)
    centre, restart = 1.0, True
    alpha_prev, beta_prev, last_step = 0.0, 1.0, 0.0
    iters = 0
    while iters < max_iter:
        x = A_vals + D
        b = g + z
        d = np.median(np.stack([-(b + lam) / a, -x, -(b - lam) / a]), axis=0)
        if iters > 0:
            last_step = float(np.max(np.abs(alpha_prev * p_prev))) if alpha_prev != 0 else 0.0
            if alpha_prev != 0.0 and last_step <= tol * np.max(np.abs(D)):
                break
            if alpha_prev == 0.0 and beta_prev == 0.0:
                break
        dd_prev = np.sum(gam * d_prev * d_prev)
        if restart or dd_prev <= 0.0:
            beta = 0.0
        else:
            beta = max(0.0, (np.sum(gam * d * d) - np.sum(gam * d * d_prev)) / dd_prev)
        restart = False
        p = d + beta * p_prev
        zp = hessian_product(W, ri, ci, p)
        C = np.sum(gam * p * zp)
        cand = centre * GRID
        # linear and l1 parts coordinate by coordinate: near the minimiser b is
        # close to -lam sign(x), and separate sums would cancel
        phi = np.array([np.sum(gam * (s * p * b + lam * l1_change(x, s * p))) + 0.5 * s * s * C
                        for s in cand])
        j = int(np.argmin(phi))
        if phi[j] < 0.0:
            alpha = float(cand[j])
            centre = alpha
        else:
            alpha = 0.0
            restart = True
        D = D + alpha * p
        z = z + alpha * zp
        p_prev, d_prev, alpha_prev, beta_prev = p, d, alpha, beta
        iters += 1
    if iters >= max_iter:
        last_step = float(np.max(np.abs(alpha_prev * p_prev))) if alpha_prev != 0 else 0.0
    # the conjugate combination and the grid step leave zeros inexact: every
    # coordinate whose own 1-D minimiser at the final Delta is zero is set to zero
    if snap:
        x = A_vals + D
        b = g + z
        zero = (-(b + lam) / a <= -x) & (-x <= -(b - lam) / a)
        D = np.where(zero, -A_vals, D)
    return D, iters, last_step
