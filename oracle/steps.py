"""Oracle (test infrastructure only): one block update of the block
coordinate-descent relaxation, step by step, from plain definitions.

Readings (each also listed with its reason in the design notes):
  * Blocks are contiguous column ranges I = [j0, j1) of size b in natural
    order, the last one short (Section 6.1 leaves the partition free and uses
    a graph clustering; contiguous ranges are one valid choice).
  * Block free set (Section 6.1, eq. (active_set_j)): a pair (r, c) with
    c in I is free when A_rc != 0 or |(S - W)_rc| > lambda; at a coarse level
    it must also lie in the level's set C_l (Section 7, eq. (MLE_l1_prior_C)).
  * Coordinates of the block problem: each unordered free pair once, as (r, c)
    with c in I and (r not in I or r <= c), ordered by column c ascending and
    then row r ascending.
  * Neighbourhood N (Section 6.1.1, eq. (extended_set)): the rows r outside I
    that appear in the block's free set, ascending (the printed set builder
    quantifies the wrong index; this is the set the text describes).
  * Newton direction: cyclic coordinate descent on the block model in that
    coordinate order, stopping after a sweep with max|mu| <= tol*max|Delta|
    or after ``max_sweeps`` sweeps.
  * Step length: the rule of ``quic_plain.linesearch_dense``.
Everything here uses the exact dense W = A^{-1}; the library reaches the same
entries with conjugate gradients, the Schur complement (App. A.1) and the
neighbour identity (App. A.2), which this module states separately and which
the tests pin against the dense definitions.
"""

from __future__ import annotations

import numpy as np

from .cd import cd_sweeps
from .core import inverse_pd, logdet_pd
from .quic_plain import linesearch_dense


def blocks(n: int, b: int):
    return [(j0, min(j0 + b, n)) for j0 in range(0, n, b)]


def cov_block(X: np.ndarray, j0: int, j1: int) -> np.ndarray:
    """S_J = X^T X_J / m, the n x |I| column block (Section 6, samples kept, S implicit)."""
    X = np.asarray(X, dtype=np.float64)
    return X.T @ X[:, j0:j1] / X.shape[0]


def inverse_columns(A: np.ndarray, cols) -> np.ndarray:
    """W_J = A^{-1} E_J, the columns J of the inverse (Section 6.1), by a dense solve."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    E = np.zeros((n, len(cols)))
    E[np.asarray(cols), np.arange(len(cols))] = 1.0
    return np.linalg.solve(A, E)


def screen(G_J, A_J, lam, j0, j1, candidates=None):
    """Free rows of every block column, ascending (eq. (active_set_j)).

    ``candidates`` (optional) maps a column c to the sorted rows allowed at
    the current level, i.e. {r : (r, c) in C_l}.
    """
    out = []
    for ci, c in enumerate(range(j0, j1)):
        mask = (A_J[:, ci] != 0) | (np.abs(G_J[:, ci]) > lam)
        rows = np.nonzero(mask)[0]
        if candidates is not None:
            rows = np.intersect1d(rows, candidates[c], assume_unique=False)
        out.append(rows.astype(np.int64))
    return out


def coordinates(free, j0, j1):
    rr, cc = [], []
    for ci, c in enumerate(range(j0, j1)):
        for r in free[ci]:
            if r < j0 or r >= j1 or r <= c:
                rr.append(int(r))
                cc.append(c)
    return np.asarray(rr, dtype=np.int64), np.asarray(cc, dtype=np.int64)


def neighborhood(free, j0, j1):
    allr = np.concatenate([f for f in free] + [np.zeros(0, dtype=np.int64)])
    allr = allr[(allr < j0) | (allr >= j1)]
    return np.unique(allr)


def local_set(j0, j1, N):
    return np.concatenate([np.arange(j0, j1, dtype=np.int64), np.asarray(N, dtype=np.int64)])


def cd_block(W, r, c, S_vals, A_vals, lam, j0, j1, N, max_sweeps=20, tol=1e-4):
    """Block Newton direction by cyclic CD (Section 6.1.1) on W restricted to J' = I u N."""
    Jp = local_set(j0, j1, N)
    loc = {int(g): k for k, g in enumerate(Jp)}
    W_JJ = np.asarray(W, dtype=np.float64)[np.ix_(Jp, Jp)]
    ri = np.array([loc[int(x)] for x in r], dtype=np.int32)
    ci = np.array([loc[int(x)] for x in c], dtype=np.int32)
    return cd_sweeps(W_JJ, ri, ci, S_vals, A_vals, lam, max_sweeps, tol)


def delta_matrix(n, r, c, vals):
    D = np.zeros((n, n))
    D[r, c] = vals
    D[c, r] = vals
    return D


def block_update(A, S, j0, j1, lam, candidates=None, max_sweeps=20, tol=1e-4, W=None):
    """One block update of Algorithm 2 (BCD-IC) with every step written out.

    Returns a dict with the intermediate quantities and the new iterate.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if W is None:
        W = inverse_pd(A)
    G_J = S[:, j0:j1] - W[:, j0:j1]
    A_J = A[:, j0:j1]
    free = screen(G_J, A_J, lam, j0, j1, candidates)
    r, c = coordinates(free, j0, j1)
    N = neighborhood(free, j0, j1)
    D_vals, sweeps, last = cd_block(W, r, c, S[r, c], A[r, c], lam, j0, j1, N,
                                    max_sweeps, tol)
    D = delta_matrix(n, r, c, D_vals)
    alpha, dF, trials = linesearch_dense(A, D, S, lam)
    A_new = A + alpha * D
    return dict(W=W, G_J=G_J, free=free, r=r, c=c, N=N, D_vals=D_vals, D=D,
                sweeps=sweeps, last_max_mu=last, alpha=alpha, dF=dF,
                trials=trials, A_new=A_new)


# --------------------------------------------------------------------------
# Schur complement route of the line search (Section 6.1.2, App. A.1)
# --------------------------------------------------------------------------

def schur_line_matrices(W_II, W_NI, W_NN, D_II, D_IN):
    """B0, B1, B2 with log det(A + a*D) = log det A_22 + log det(B0 + a B1 + a^2 B2).

    D is zero outside the rows/columns I and its off-block part lives in the
    columns N.  With M = D_IN W_NI (eq. (T) uses T = M B0):
        B0 = W_II^{-1}                                   (eq. (B_0))
        B1 = D_II + M B0 + B0 M^T                        (text after eq. (computingBi2))
        B2 = -D_IN W_NN D_NI + M B0 M^T
    The last line follows from B2 = -D_12 A_22^{-1} D_21 and eq. (A22),
    A_22^{-1} = W_22 - W_21 B0 W_12; the printed eq. (A22_detailed) has the
    opposite sign on the first term and transposes D_12, and the printed
    eq. (computingBi3) has the opposite sign on its correction term (block
    inversion gives W_22 = A_22^{-1} + A_22^{-1} A_21 W_11 A_12 A_22^{-1}).
    """
    B0 = np.linalg.inv(W_II)
    B0 = 0.5 * (B0 + B0.T)
    M = D_IN @ W_NI
    B1 = D_II + M @ B0 + B0 @ M.T
    B2 = -D_IN @ W_NN @ D_IN.T + M @ B0 @ M.T
    return B0, B1, B2


def schur_logdet_change(B0, B1, B2, alpha):
    """log det(A + alpha*D) - log det(A), or None if A + alpha*D is not PD (eq. (Schurs_PDness))."""
    ld1 = logdet_pd(B0 + alpha * B1 + alpha * alpha * B2)
    if ld1 is None:
        return None
    return ld1 - logdet_pd(B0)


def w_block_from_neighbors(A_II, A_IN, W_NI):
    """W_II = A_II^{-1} (I - K), K = A_IN W_NI  (App. A.2, eqs. (reducingGradients1/2))."""
    b = A_II.shape[0]
    return np.linalg.solve(A_II, np.eye(b) - A_IN @ W_NI)


# --------------------------------------------------------------------------
# multilevel hierarchy (Section 3.2, Section 7)
# --------------------------------------------------------------------------

def hierarchy(supp_keys, free_keys, free_absg):
    """Nested sets C_1 ... C_L as prefix lengths of one ranking.

    Ranking: the support first (keys ascending), then the free pairs outside
    the support by |g| descending, ties by key ascending.  Sizes:
    |C_1| = max(ceil(|F|/2), |supp|), |C_{l+1}| = max(ceil(|C_l|/2), |supp|),
    stopping at the first level equal to |supp| (Section 7, incl. footnote;
    Section 3.2). |F| counts unordered pairs of F u supp.
    Returns (ranking keys, [|C_1|, ..., |C_L|]).
    """
    supp = np.unique(np.asarray(supp_keys, dtype=np.int64))
    fk = np.asarray(free_keys, dtype=np.int64)
    fg = np.asarray(free_absg, dtype=np.float64)
    keep = ~np.isin(fk, supp)
    rk, rg = fk[keep], fg[keep]
    # unique keys (callers pass unique keys already)
    order = np.lexsort((rk, -rg))
    ranking = np.concatenate([supp, rk[order]])
    nf = ranking.size
    ns = supp.size
    sizes = [max(-(-nf // 2), ns)]
    while sizes[-1] != ns:
        sizes.append(max(-(-sizes[-1] // 2), ns))
    return ranking, sizes


def level_candidates(ranking, size, n):
    """Per-column candidate rows {r : (r, c) in C_l} for the first ``size`` ranked pairs."""
    keys = ranking[:size]
    i = keys // n
    j = keys % n
    rows = np.concatenate([i, j])
    cols = np.concatenate([j, i])
    cand = {c: [] for c in range(n)}
    order = np.lexsort((rows, cols))
    rows, cols = rows[order], cols[order]
    out = {}
    starts = np.searchsorted(cols, np.arange(n + 1))
    for c in range(n):
        out[c] = np.unique(rows[starts[c]:starts[c + 1]])
    del cand
    return out
