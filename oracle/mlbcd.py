"""Oracle (test infrastructure only): the multilevel cycle of Algorithm 1 with
the block relaxation of Algorithm 2, for small n (dense W at every block).

  * relaxation = one sweep of block updates over the blocks in order
    (Algorithm 2, one outer iteration), restricted at level l to C_l;
  * one relaxation per level, the coarsest included (Section 7, nu = nu_c = 1);
  * the hierarchy comes from the free set and gradient recorded during the
    previous cycle's finest sweep; the first cycle uses the free set
    {|S_ij| > lambda} u supp(A0) with |g| = |S_ij| off the diagonal
    (Section 7 and its footnote), A0 = I (Section 8);
  * a free pair's |g| is the one seen at its latest free screening in the
    sweep; the hierarchy uses the support of the iterate at the start of the
    cycle;
  * convergence: the finest sweep's max-norm of the min-norm subgradient,
    each block measured before its own update (Section 3.2: the fine
    relaxation monitors convergence).
"""

from __future__ import annotations

import numpy as np

from .core import covariance, inverse_pd, min_norm_subgradient, objective
from .steps import block_update, blocks, hierarchy, level_candidates


def relax(A, S, lam, b, candidates=None, max_sweeps=20, tol=1e-4):
    """One block-coordinate sweep; returns (A, records, kkt_max, kkt_l1, per-block log)."""
    n = A.shape[0]
    records = {}
    seq = 0
    kmax, kl1 = 0.0, 0.0
    log = []
    for (j0, j1) in blocks(n, b):
        out = block_update(A, S, j0, j1, lam, candidates, max_sweeps, tol)
        G_J = out["G_J"]
        m = min_norm_subgradient(G_J, A[:, j0:j1], lam)
        kmax = max(kmax, float(np.max(np.abs(m))))
        kl1 += float(np.sum(np.abs(m)))
        for ci, c in enumerate(range(j0, j1)):
            for r in out["free"][ci]:
                i, j = (int(r), c) if r <= c else (c, int(r))
                records[i * n + j] = (abs(G_J[r, ci]), seq)
                seq += 1
        log.append(dict(j0=j0, j1=j1, alpha=out["alpha"], dF=out["dF"],
                        ncoord=int(out["r"].size), nN=int(out["N"].size)))
        A = out["A_new"]
    return A, records, kmax, kl1, log


def supp_keys(A):
    n = A.shape[0]
    i, j = np.nonzero(np.triu(A != 0))
    return np.sort(i.astype(np.int64) * n + j)


def solve(X=None, lam=0.1, b=32, tol=1e-6, max_cycles=50, S=None, multilevel=True,
          max_sweeps=20, cd_tol=1e-4):
    """ML-BCD on a dense iterate. Returns (A, info with per-cycle history)."""
    if S is None:
        S = covariance(X)
    n = S.shape[0]
    A = np.eye(n)
    iu, ju = np.nonzero(np.triu(np.abs(S) > lam, 1))
    fkeys = iu.astype(np.int64) * n + ju
    fg = np.abs(S[iu, ju])
    hist = []
    kmax = np.inf
    for cyc in range(max_cycles):
        levels = []
        if multilevel:
            ranking, sizes = hierarchy(supp_keys(A), fkeys, fg)
            for size in reversed(sizes):
                cand = level_candidates(ranking, size, n)
                A, _, _, _, _ = relax(A, S, lam, b, cand, max_sweeps, cd_tol)
                levels.append(size)
        A, rec, kmax, kl1, _ = relax(A, S, lam, b, None, max_sweeps, cd_tol)
        fkeys = np.fromiter(rec.keys(), dtype=np.int64, count=len(rec))
        fg = np.array([rec[k][0] for k in fkeys])
        hist.append(dict(cycle=cyc, levels=levels, F=objective(A, S, lam), kkt_sweep=kmax,
                         kkt_l1=kl1, nnz=int(np.count_nonzero(A))))
        if kmax <= tol:
            break
    W = inverse_pd(A)
    kkt_final = float(np.max(np.abs(min_norm_subgradient(S - W, A, lam))))
    return A, dict(history=hist, kkt_final=kkt_final, objective=objective(A, S, lam))
