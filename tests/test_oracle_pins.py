"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test ties an oracle function to something other than itself: closed
forms, the optimality condition, brute-force enumeration, exact algebraic
identities, or a brute-force 1-D minimisation.
"""

import numpy as np
import pytest
import scipy.optimize as so

from oracle import bruteforce, core, mlbcd, quic_plain, steps
from oracle.cd import cd_sweeps


def _samples(n, m, seed):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((n, n)) * 0.3
    Sig = C @ C.T + np.eye(n)
    L = np.linalg.cholesky(Sig)
    return rng.standard_normal((m, n)) @ L.T


def _kkt_certificate(A, S, lam, tol):
    W = np.linalg.inv(A)
    G = S - W
    on = A != 0
    assert np.all(np.abs(G[~on]) <= lam + tol)
    assert np.all(np.abs(G[on] + lam * np.sign(A[on])) <= tol)
    assert np.allclose(A, A.T, atol=0, rtol=0)
    assert np.all(np.linalg.eigvalsh(A) > 0)


# ---------------------------------------------------------------- closed forms

def test_diagonal_regime_closed_form():
    # lam >= max off-diagonal |S_ij| gives A* = diag(1 / (S_ii + lam))  (diagonal penalised)
    X = _samples(6, 40, 1)
    S = core.covariance(X)
    off = np.abs(S - np.diag(np.diag(S))).max()
    lam = off * 1.01
    A, info = quic_plain.solve(S, lam, tol=1e-13)
    np.testing.assert_allclose(A, np.diag(1.0 / (np.diag(S) + lam)), rtol=1e-12, atol=1e-14)
    A2, _ = mlbcd.solve(S=S, lam=lam, b=4, tol=1e-12)
    np.testing.assert_allclose(A2, np.diag(1.0 / (np.diag(S) + lam)), rtol=1e-12, atol=1e-14)


def test_lambda_zero_gives_inverse_covariance():
    X = _samples(7, 60, 2)
    S = core.covariance(X)
    A, info = quic_plain.solve(S, 0.0, tol=1e-12)
    np.testing.assert_allclose(A, np.linalg.inv(S), rtol=1e-9, atol=1e-10)


def test_one_variable():
    S = np.array([[1.7]])
    A, _ = quic_plain.solve(S, 0.3, tol=1e-14)
    assert A[0, 0] == pytest.approx(1.0 / 2.0, rel=1e-13)


@pytest.mark.parametrize("s12,lam", [(0.6, 0.2), (-0.6, 0.2), (0.1, 0.2)])
def test_two_variables_closed_form(s12, lam):
    S = np.array([[1.3, s12], [s12, 0.9]])
    if abs(s12) > lam:
        W = np.array([[1.3 + lam, s12 - lam * np.sign(s12)],
                      [s12 - lam * np.sign(s12), 0.9 + lam]])
        expect = np.linalg.inv(W)
    else:
        expect = np.diag(1.0 / (np.diag(S) + lam))
    A, _ = quic_plain.solve(S, lam, tol=1e-14)
    np.testing.assert_allclose(A, expect, rtol=1e-11, atol=1e-13)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("n,lam,seed", [(3, 0.15, 3), (4, 0.12, 4), (4, 0.3, 5)])
def test_bruteforce_support_enumeration(n, lam, seed):
    X = _samples(n, 30, seed)
    S = core.covariance(X)
    Ab = bruteforce.solve(S, lam)
    Aq, _ = quic_plain.solve(S, lam, tol=1e-13)
    Am, _ = mlbcd.solve(S=S, lam=lam, b=2, tol=1e-12)
    np.testing.assert_allclose(Aq, Ab, atol=1e-8)
    np.testing.assert_allclose(Am, Ab, atol=1e-8)
    assert np.array_equal(Aq != 0, np.abs(Ab) > 1e-10)
    assert np.array_equal(Am != 0, np.abs(Ab) > 1e-10)


# ---------------------------------------------------------------- optimality

def test_kkt_certificate_and_diag_identity():
    from synth import workload
    X, P, spec = workload("chain_n64_m48")
    S = core.covariance(X)
    lam = spec["lam"]
    A, info = quic_plain.solve(S, lam, tol=1e-12)
    _kkt_certificate(A, S, lam, 1e-10)
    W = np.linalg.inv(A)
    np.testing.assert_allclose(np.diag(W), np.diag(S) + lam, atol=1e-10)


def test_ml_bcd_matches_solution_oracle():
    from synth import workload
    X, P, spec = workload("chain_n64_m48")
    S = core.covariance(X)
    lam = spec["lam"]
    Aq, _ = quic_plain.solve(S, lam, tol=1e-12)
    Am, info = mlbcd.solve(S=S, lam=lam, b=spec["block"], tol=1e-10)
    assert np.array_equal(Aq != 0, Am != 0)
    assert abs(info["objective"] - core.objective(Aq, S, lam)) <= 1e-10 * abs(info["objective"])
    # monotone cycles (multilevel cycle with a monotone relaxation, Section 4.2)
    Fs = [h["F"] for h in info["history"]]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(Fs, Fs[1:]))


# ---------------------------------------------------------------- coordinate descent

def _model(D, S, W, A, lam):
    """Block model: tr(D(S-W)) + 0.5 tr(DWDW) + lam*||A+D||_1 (eq. (Quad_MLE_l1_prior))."""
    return np.sum(D * (S - W)) + 0.5 * np.trace(D @ W @ D @ W) + lam * np.sum(np.abs(A + D))


@pytest.mark.parametrize("i,k", [(0, 2), (1, 1), (3, 0)])
def test_single_coordinate_step_is_1d_argmin(i, k):
    rng = np.random.default_rng(7)
    nj = 4
    B = rng.standard_normal((nj, nj))
    W = B @ B.T + nj * np.eye(nj)
    S = rng.standard_normal((nj, nj)); S = S + S.T
    A = rng.standard_normal((nj, nj)) * 0.3; A = A + A.T
    A[i, k] = A[k, i] = 0.05
    lam = 0.4
    D, sweeps, _ = cd_sweeps(W, [i], [k], [S[i, k]], [A[i, k]], lam, 1, 0.0)
    E = np.zeros((nj, nj)); E[i, k] = E[k, i] = 1.0
    phi = lambda mu: _model(mu * E, S, W, A, lam)
    res = so.minimize_scalar(phi, bounds=(-10, 10), method="bounded",
                             options=dict(xatol=1e-12))
    # phi is piecewise quadratic: check against the exact kink too
    cands = [res.x, -A[i, k]]
    best = min(cands, key=phi)
    assert D[0] == pytest.approx(best, abs=1e-8)
    assert phi(D[0]) <= phi(best) + 1e-12


def test_cd_converges_to_model_kkt():
    rng = np.random.default_rng(8)
    nj = 6
    B = rng.standard_normal((nj, nj))
    W = B @ B.T / nj + np.eye(nj)
    S = rng.standard_normal((nj, nj)) * 0.5; S = S + S.T
    A = rng.standard_normal((nj, nj)) * 0.2; A = (A + A.T) * (rng.random((nj, nj)) < 0.5)
    A = np.triu(A) + np.triu(A, 1).T
    lam = 0.3
    ri, ci = np.triu_indices(nj)
    D, sweeps, _ = cd_sweeps(W, ri, ci, S[ri, ci], A[ri, ci], lam, 2000, 0.0)
    Dm = np.zeros((nj, nj)); Dm[ri, ci] = D; Dm[ci, ri] = D
    Gt = S - W + W @ Dm @ W
    X = A + Dm
    on = X != 0
    assert np.all(np.abs(Gt[on] + lam * np.sign(X[on])) <= 1e-10)
    assert np.all(np.abs(Gt[~on]) <= lam + 1e-10)


def _model_block(seed, nj=8, lam=0.3):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((nj, nj))
    W = B @ B.T / nj + np.eye(nj)
    S = rng.standard_normal((nj, nj)) * 0.5; S = S + S.T
    A = rng.standard_normal((nj, nj)) * 0.2; A = (A + A.T) * (rng.random((nj, nj)) < 0.5)
    A = np.triu(A) + np.triu(A, 1).T
    ri, ci = np.triu_indices(nj)
    return W, S, A, ri, ci, lam


@pytest.mark.parametrize("seed", [8, 9, 10])
def test_pcd_cg_converges_to_the_cd_minimiser(seed):
    """PCD-CG and cyclic CD minimise the same strictly convex block model: run
    to convergence they meet at its unique minimiser (checked by its KKT)."""
    from oracle import pcd
    W, S, A, ri, ci, lam = _model_block(seed)
    Dc, _, _ = cd_sweeps(W, ri, ci, S[ri, ci], A[ri, ci], lam, 5000, 0.0)
    Dp, its, _ = pcd.pcd_cg(W, ri, ci, S[ri, ci], A[ri, ci], lam, max_iter=3000, tol=1e-13)
    assert its > 3
    assert np.max(np.abs(Dp - Dc)) <= 1e-8 * max(1.0, np.max(np.abs(Dc)))
    Dm = np.zeros_like(W); Dm[ri, ci] = Dp; Dm[ci, ri] = Dp
    Gt = S - W + W @ Dm @ W
    X = A + Dm
    on = X != 0
    assert np.all(np.abs(Gt[on] + lam * np.sign(X[on])) <= 1e-7)
    assert np.all(np.abs(Gt[~on]) <= lam + 1e-7)


def test_pcd_first_step_is_the_grid_minimiser_of_the_model():
    """One PCD-CG iteration from Delta = 0: p is every coordinate's own 1-D
    minimiser (brute force, independent of the closed form), and the step is
    the candidate with the smallest model value evaluated directly with dense
    matrices (independent of the B, C, l1 split the iteration uses)."""
    from oracle import pcd
    W, S, A, ri, ci, lam = _model_block(11, nj=7)
    Sv, Av = S[ri, ci], A[ri, ci]
    D1, its, _ = pcd.pcd_cg(W, ri, ci, Sv, Av, lam, max_iter=1, tol=0.0, snap=False)
    assert its == 1
    p = np.empty(ri.size)
    for k in range(ri.size):
        def f(mu, k=k):
            e = np.zeros(ri.size); e[k] = mu
            return pcd.block_model(W, ri, ci, Sv, Av, lam, e)
        r = so.minimize_scalar(f, bracket=(-3, 3), tol=1e-14)
        p[k] = r.x
    vals = [pcd.block_model(W, ri, ci, Sv, Av, lam, s * p) for s in pcd.GRID]
    best = pcd.GRID[int(np.argmin(vals))]
    assert min(vals) < pcd.block_model(W, ri, ci, Sv, Av, lam, 0 * p)
    assert np.max(np.abs(D1 - best * p)) <= 1e-6 * max(1.0, np.max(np.abs(p)))


# ---------------------------------------------------------------- Schur route, App. A

def _structured(seed, n=12, I=(0, 1, 2, 3), N=(5, 7, 9)):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n)) * 0.3
    A = B @ B.T + n * 0.2 * np.eye(n)
    I = np.array(I); N = np.array(N)
    D = np.zeros((n, n))
    blk = rng.standard_normal((len(I), len(I))) * 0.3
    D[np.ix_(I, I)] = blk + blk.T
    cross = rng.standard_normal((len(I), len(N))) * 0.3
    D[np.ix_(I, N)] = cross
    D[np.ix_(N, I)] = cross.T
    return A, D, I, N


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_schur_line_matrices_match_direct_logdet(seed):
    A, D, I, N = _structured(seed)
    W = np.linalg.inv(A)
    B0, B1, B2 = steps.schur_line_matrices(W[np.ix_(I, I)], W[np.ix_(N, I)], W[np.ix_(N, N)],
                                           D[np.ix_(I, I)], D[np.ix_(I, N)])
    for a in (1.0, 0.5, 0.25, 0.125):
        direct = core.logdet_pd(A + a * D)
        via = steps.schur_logdet_change(B0, B1, B2, a)
        if direct is None:
            assert via is None
        else:
            assert via == pytest.approx(direct - core.logdet_pd(A), abs=1e-10)


def test_printed_b2_sign_would_be_wrong():
    A, D, I, N = _structured(3)
    W = np.linalg.inv(A)
    B0, B1, B2 = steps.schur_line_matrices(W[np.ix_(I, I)], W[np.ix_(N, I)], W[np.ix_(N, N)],
                                           D[np.ix_(I, I)], D[np.ix_(I, N)])
    Dn = D[np.ix_(I, N)]
    printed = B2 + 2 * Dn @ W[np.ix_(N, N)] @ Dn.T   # first term with the printed sign
    direct = core.logdet_pd(A + 0.5 * D) - core.logdet_pd(A)
    wrong = steps.schur_logdet_change(B0, B1, printed, 0.5)
    assert wrong is None or abs(wrong - direct) > 1e-6


def test_neighbour_identity_app_a2():
    rng = np.random.default_rng(11)
    n = 14
    I = np.arange(0, 4)
    N = np.array([6, 9, 12])
    B = rng.standard_normal((n, n)) * 0.2
    A = B @ B.T
    rest = np.setdiff1d(np.arange(n), np.concatenate([I, N]))
    A[np.ix_(I, rest)] = 0.0
    A[np.ix_(rest, I)] = 0.0
    A += n * 0.3 * np.eye(n)
    W = np.linalg.inv(A)
    Wii = steps.w_block_from_neighbors(A[np.ix_(I, I)], A[np.ix_(I, N)], W[np.ix_(N, I)])
    np.testing.assert_allclose(Wii, W[np.ix_(I, I)], atol=1e-12)


def test_logdet_identity_plus_keeps_small_terms():
    rng = np.random.default_rng(5)
    n = 300
    B = rng.standard_normal((n, n))
    E = 0.1 * (B + B.T) / np.sqrt(n)
    assert core.logdet_identity_plus(E) == pytest.approx(np.linalg.slogdet(np.eye(n) + E)[1],
                                                        abs=1e-11)
    E = 1e-10 * (B + B.T)
    series = np.trace(E) - 0.5 * np.sum(E * E)
    assert core.logdet_identity_plus(E) == pytest.approx(series, rel=1e-12)
    assert core.logdet_identity_plus(-2 * np.eye(3)) is None


def test_objective_change_matches_difference():
    A, D, I, N = _structured(4)
    S = _structured(5)[0] / 3
    lam = 0.2
    dF = quic_plain.objective_change(A, D, S, lam)
    for a in (1.0, 0.5, 0.1):
        ref = core.objective(A + a * D, S, lam) - core.objective(A, S, lam)
        if np.isfinite(ref):
            assert dF(a) == pytest.approx(ref, abs=1e-10)


def test_linesearch_skips_non_pd_trials():
    A = np.eye(3)
    D = np.diag([-1.5, 0.0, 0.0])            # alpha = 1 makes A singular-negative
    S = np.eye(3) * 2.0
    alpha, dF, trials = quic_plain.linesearch_dense(A, D, S, 0.0)
    # F(alpha) along the line: -log(1 - 1.5a) - 3a; minimiser a = 1/3 - ... ; 0.25 is the best trial
    vals = {a: -np.log(1 - 1.5 * a) - 3 * a for a in (0.5, 0.25, 0.125)}
    assert alpha == min(vals, key=vals.get)
    assert dF == pytest.approx(min(vals.values()), abs=1e-14)


# ---------------------------------------------------------------- hierarchy

def test_hierarchy_sizes_and_order():
    n = 10
    supp = [0 * n + 0, 1 * n + 1, 2 * n + 5]
    free = [2 * n + 5, 0 * n + 3, 1 * n + 4, 3 * n + 7, 4 * n + 9, 6 * n + 8, 0 * n + 9]
    g = [0.0, 0.5, 0.9, 0.5, 0.2, 0.7, 0.3]
    ranking, sizes = steps.hierarchy(supp, free, g)
    # |F u supp| = 9 pairs -> |C_1| = max(5, 3) = 5 -> |C_2| = 3 = |supp|
    assert sizes == [5, 3]
    assert list(ranking[:3]) == sorted(supp)
    # |g| descending, ties by key ascending: 0.9(14) 0.7(68) 0.5(3) 0.5(37) 0.3(9) 0.2(49)
    assert list(ranking[3:]) == [14, 68, 3, 37, 9, 49]


def test_hierarchy_nested_and_terminates():
    rng = np.random.default_rng(3)
    supp = np.arange(0, 40) * 101
    free = np.arange(40, 1000) * 7 + 5
    g = rng.random(free.size)
    ranking, sizes = steps.hierarchy(supp, free, g)
    nf = np.union1d(supp, free).size
    assert sizes[0] == max(-(-nf // 2), supp.size)
    assert ranking.size == nf
    assert all(a >= b for a, b in zip(sizes, sizes[1:]))
    assert sizes[-1] == supp.size
    for a, b in zip(sizes, sizes[1:]):
        assert b == max(-(-a // 2), supp.size)


# ---------------------------------------------------------------- relaxation properties

def test_block_updates_are_monotone():
    from synth import workload
    X, P, spec = workload("grid_n400_m300")
    S = core.covariance(X)
    lam = spec["lam"]
    A = np.eye(S.shape[0])
    F0 = core.objective(A, S, lam)
    A1, rec, kmax, kl1, log = mlbcd.relax(A, S, lam, spec["block"])
    assert all(entry["dF"] <= 0.0 for entry in log)
    F1 = core.objective(A1, S, lam)
    assert F1 - F0 == pytest.approx(sum(e["dF"] for e in log), abs=1e-9)


def test_coarse_solution_correspondence():
    """Lemma of Section 4.2: a level C containing supp(A*) has A* as its solution."""
    from synth import workload
    X, P, spec = workload("chain_n64_m48")
    S = core.covariance(X)
    lam = spec["lam"]
    Astar, _ = quic_plain.solve(S, lam, tol=1e-12)
    n = S.shape[0]
    keys = core.support_pairs(Astar)
    cand = steps.level_candidates(keys, keys.size, n)
    A = np.eye(n)
    for _ in range(12):
        A, _, _, _, _ = mlbcd.relax(A, S, lam, spec["block"], cand, max_sweeps=50, tol=1e-10)
    np.testing.assert_allclose(A, Astar, atol=1e-8)


# ---------------------------------------------------------------- covariance (Section 5, S = X^T X / m)

def test_covariance_hand_worked_example():
    """m = 2 samples of n = 3 variables, worked out by hand: S = X^T X / m
    with no centring and the divisor m (not m - 1)."""
    X = np.array([[1.0, 2.0, 0.0],
                  [3.0, -1.0, 2.0]])
    expect = np.array([[5.0, -0.5, 3.0],
                       [-0.5, 2.5, -1.0],
                       [3.0, -1.0, 2.0]])
    np.testing.assert_array_equal(core.covariance(X), expect)
    np.testing.assert_array_equal(steps.cov_block(X, 1, 3), expect[:, 1:3])


def test_covariance_entries_by_loops_and_structure():
    rng = np.random.default_rng(21)
    m, n = 7, 5
    X = rng.standard_normal((m, n)) + 3.0     # a non-zero mean: centring would change S
    S = core.covariance(X)
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for t in range(m):
                acc += X[t, i] * X[t, j]
            assert S[i, j] == pytest.approx(acc / m, rel=1e-14)
    # diag S = ||X_{:,i}||^2 / m, and S is symmetric
    for i in range(n):
        assert S[i, i] == pytest.approx(sum(v * v for v in X[:, i]) / m, rel=1e-14)
    assert np.array_equal(S, S.T)
    # a constant column c gives S_ii = c^2 (the centred estimate would give 0)
    Xc = X.copy()
    Xc[:, 2] = 1.5
    assert core.covariance(Xc)[2, 2] == pytest.approx(2.25, rel=1e-15)


def test_cov_block_rows_by_loops_and_symmetric_diagonal_block():
    rng = np.random.default_rng(22)
    m, n, j0, j1 = 9, 8, 3, 6
    X = rng.standard_normal((m, n))
    SJ = steps.cov_block(X, j0, j1)
    assert SJ.shape == (n, j1 - j0)
    for i in range(n):
        for c in range(j0, j1):
            acc = sum(X[t, i] * X[t, c] for t in range(m))
            assert SJ[i, c - j0] == pytest.approx(acc / m, rel=1e-13, abs=1e-15)
    SII = SJ[j0:j1, :]
    np.testing.assert_allclose(SII, SII.T, rtol=1e-15, atol=0)
    for c in range(j0, j1):
        assert SJ[c, c - j0] == pytest.approx(np.sum(X[:, c] ** 2) / m, rel=1e-14)


# ---------------------------------------------------------------- log det, in high precision

mpmath = pytest.importorskip("mpmath")


def _mp_logdet(M, dps=60):
    """log det of a symmetric matrix by an mpmath Cholesky at `dps` digits
    (None when a pivot is not positive)."""
    with mpmath.workdps(dps):
        A = mpmath.matrix([[mpmath.mpf(float(v)) for v in row] for row in M])
        return _mp_logdet_matrix(A)


def _mp_logdet_matrix(A):
    n = A.rows
    L = mpmath.matrix(n, n)
    total = mpmath.mpf(0)
    for j in range(n):
        s = A[j, j] - sum(L[j, k] ** 2 for k in range(j))
        if s <= 0:
            return None
        L[j, j] = mpmath.sqrt(s)
        total += mpmath.log(s)
        for i in range(j + 1, n):
            L[i, j] = (A[i, j] - sum(L[i, k] * L[j, k] for k in range(j))) / L[j, j]
    return total


def _mp_objective_change(A, D, S, lam, alpha, dps=60):
    """F(A + alpha D) - F(A) at `dps` digits, every term from its definition
    (eq. (MLE_l1_prior)): the log dets by Cholesky, the trace and the l1 norm
    entry by entry."""
    n = A.shape[0]
    with mpmath.workdps(dps):
        a = mpmath.mpf(float(alpha))
        Am = mpmath.matrix([[mpmath.mpf(float(v)) for v in row] for row in A])
        Dm = mpmath.matrix([[mpmath.mpf(float(v)) for v in row] for row in D])
        Bm = Am + a * Dm
        l0, l1 = _mp_logdet_matrix(Am), _mp_logdet_matrix(Bm)
        if l1 is None:
            return None
        tr = sum(mpmath.mpf(float(S[i, j])) * Dm[i, j] for i in range(n) for j in range(n))
        l1n = sum(abs(Bm[i, j]) - abs(Am[i, j]) for i in range(n) for j in range(n))
        return float(-(l1 - l0) + a * tr + mpmath.mpf(float(lam)) * l1n)


@pytest.mark.parametrize("scale", [1e-12, 1e-9, 1e-6, 1e-3, 0.3])
def test_logdet_identity_plus_against_high_precision(scale):
    """log det(I + E) by the blocked log1p Cholesky (block 4 on n = 12, so the
    trailing update between blocks runs) against a 60-digit Cholesky."""
    rng = np.random.default_rng(31)
    n = 12
    B = rng.standard_normal((n, n))
    E = scale * (B + B.T) / np.sqrt(n)
    ref = float(_mp_logdet_exact_shift(E))
    for blk in (4, 128):
        got = core.logdet_identity_plus(E, block=blk)
        assert got == pytest.approx(ref, rel=1e-12, abs=1e-300)


def _mp_logdet_exact_shift(E, dps=80):
    """log det(I + E) with I + E formed exactly in mpmath (float64 would round
    the small entries of E away)."""
    n = E.shape[0]
    with mpmath.workdps(dps):
        M = mpmath.matrix([[mpmath.mpf(float(E[i, j])) + (1 if i == j else 0) for j in range(n)]
                           for i in range(n)])
        return _mp_logdet_matrix(M)


@pytest.mark.parametrize("step", [1e-12, 1e-9, 1e-6, 1e-3])
def test_objective_change_against_high_precision(step):
    """The line search's F(A + alpha D) - F(A) (whitened log det, term-wise l1
    change) at alpha ||D|| from 1e-12 to 1e-3 against the plain definition
    evaluated at 60 digits."""
    A, D, I, N = _structured(6)
    S = _structured(7)[0] / 3
    A[0, 5] = A[5, 0] = 0.0          # a zero entry of A under the direction: sign change
    lam = 0.2
    dF = quic_plain.objective_change(A, D, S, lam)
    nd = np.max(np.abs(D))
    for alpha in (step / nd, 0.5 * step / nd):
        ref = _mp_objective_change(A, D, S, lam, alpha)
        got = dF(alpha)
        assert got == pytest.approx(ref, rel=1e-9, abs=1e-14 * step)


def test_logdet_pd_and_cholesky_closed_forms():
    M = np.array([[4.0, 2.0], [2.0, 5.0]])     # L = [[2, 0], [1, 2]], det 16
    L = core.cholesky_lower(M)
    np.testing.assert_allclose(L, [[2.0, 0.0], [1.0, 2.0]], rtol=1e-15)
    assert core.logdet_pd(M) == pytest.approx(np.log(16.0), rel=1e-15)
    assert core.logdet_pd(np.array([[1.0, 2.0], [2.0, 1.0]])) is None
    assert core.cholesky_lower(np.array([[-1.0]])) is None


def test_inverse_pd_is_an_inverse():
    A, _, _, _ = _structured(8)
    W = core.inverse_pd(A)
    np.testing.assert_allclose(A @ W, np.eye(A.shape[0]), atol=1e-12)
    np.testing.assert_array_equal(W, W.T)
    with pytest.raises(np.linalg.LinAlgError):
        core.inverse_pd(np.array([[1.0, 2.0], [2.0, 1.0]]))


def test_objective_closed_form_and_gradient_by_differences():
    # diagonal A: F = -sum log a_i + sum S_ii a_i + lam sum a_i
    S = np.array([[2.0, 0.3], [0.3, 1.0]])
    A = np.diag([0.5, 2.0])
    lam = 0.1
    expect = -(np.log(0.5) + np.log(2.0)) + 2.0 * 0.5 + 1.0 * 2.0 + lam * 2.5
    assert core.objective(A, S, lam) == pytest.approx(expect, rel=1e-15)
    assert core.objective(-A, S, lam) == float("inf")
    # gradient of the smooth part f(A) = -log det A + tr(SA), by central
    # differences of f along symmetric unit directions, at 60 digits
    A2, _, _, _ = _structured(9, n=5, I=(0, 1), N=(3,))
    S2 = _structured(10, n=5, I=(0, 1), N=(3,))[0] / 4
    G = core.gradient(A2, S2)
    h = 1e-20
    for (i, j) in [(0, 0), (1, 3), (2, 4), (4, 4)]:
        E = np.zeros((5, 5)); E[i, j] = E[j, i] = 1.0
        with mpmath.workdps(60):
            hp = mpmath.mpf(h)
            def f(sign):
                M = mpmath.matrix([[mpmath.mpf(float(A2[r, c])) + sign * hp * E[r, c]
                                    for c in range(5)] for r in range(5)])
                tr = sum(mpmath.mpf(float(S2[r, c])) * M[c, r] for r in range(5) for c in range(5))
                return -_mp_logdet_matrix(M) + tr
            deriv = float((f(1) - f(-1)) / (2 * hp))
        expect = G[i, j] if i == j else 2.0 * G[i, j]
        assert expect == pytest.approx(deriv, rel=1e-10, abs=1e-13)


def test_min_norm_subgradient_by_brute_force():
    """The subdifferential of lam|a| at a = 0 is [-lam, lam]; the min-norm
    element is found here by scanning it on a fine grid (Section 4,
    eq. (subgradient1))."""
    lam = 0.3
    G = np.array([[0.5, -0.1, 0.45], [-0.1, -0.8, 0.2], [0.45, 0.2, 0.05]])
    A = np.array([[1.0, 0.0, -0.2], [0.0, 2.0, 0.0], [-0.2, 0.0, 1.5]])
    m = core.min_norm_subgradient(G, A, lam)
    t = np.linspace(-1.0, 1.0, 200001)
    for i in range(3):
        for j in range(3):
            if A[i, j] != 0:
                expect = G[i, j] + lam * np.sign(A[i, j])
            else:
                cands = G[i, j] + lam * t
                expect = cands[np.argmin(np.abs(cands))]
            assert m[i, j] == pytest.approx(expect, abs=1e-5)
    assert core.kkt_max(G, A, lam) == pytest.approx(np.max(np.abs(m)), rel=1e-15)
    assert core.kkt_l1(G, A, lam) == pytest.approx(np.sum(np.abs(m)), rel=1e-15)
    # at a KKT point the measure is zero
    assert core.kkt_max(np.array([[-0.3]]), np.array([[1.0]]), 0.3) == 0.0


def test_free_mask_and_support_pairs_hand_worked():
    lam = 0.3
    G = np.array([[0.1, 0.31, -0.3], [0.31, 0.0, -0.5], [-0.3, -0.5, 0.2]])
    A = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    F = core.free_mask(G, A, lam)
    expect = np.array([[1, 1, 0], [1, 1, 1], [0, 1, 1]], dtype=bool)   # |g| = lam is not free
    np.testing.assert_array_equal(F, expect)
    A2 = np.array([[1.0, 0.0, -0.2], [0.0, 2.0, 0.0], [-0.2, 0.0, 1.5]])
    np.testing.assert_array_equal(core.support_pairs(A2), [0 * 3 + 0, 0 * 3 + 2, 1 * 3 + 1, 2 * 3 + 2])


def test_abs_change_and_l1_change_exact_cases():
    from oracle import pcd
    a = np.array([1.0, -1.0, 0.0, 0.5, -0.5, 1e16])
    d = np.array([-3.0, 0.25, -0.7, -0.5, 1.5, 1.0])
    expect = np.abs(a + d) - np.abs(a)
    expect[-1] = 1.0                     # no sign change: +d exactly, which a + d would round
    np.testing.assert_array_equal(quic_plain.abs_change(a, d), expect)
    np.testing.assert_array_equal(pcd.l1_change(a, d), expect)


# ---------------------------------------------------------------- block steps by hand

def test_block_sets_hand_worked():
    """Free rows per block column, the coordinates and the neighbourhood of
    one block on a 6-variable example written out by hand (eq. (active_set_j),
    eq. (extended_set))."""
    lam = 0.3
    n, j0, j1 = 6, 2, 4
    G = np.zeros((n, n))
    A = np.eye(n)
    G[0, 2] = 0.5     # row 0 free in column 2 (outside I)
    G[3, 2] = -0.4    # row 3 free in column 2 (inside I, below the diagonal: not a coordinate)
    G[5, 3] = 0.31    # row 5 free in column 3
    G[1, 3] = 0.3     # |g| = lam: not free
    A[4, 3] = 0.2     # non-zero in A: free whatever g is
    G_J, A_J = G[:, j0:j1], A[:, j0:j1]
    free = steps.screen(G_J, A_J, lam, j0, j1)
    assert [list(f) for f in free] == [[0, 2, 3], [3, 4, 5]]
    r, c = steps.coordinates(free, j0, j1)
    assert list(zip(r.tolist(), c.tolist())) == [(0, 2), (2, 2), (3, 3), (4, 3), (5, 3)]
    N = steps.neighborhood(free, j0, j1)
    assert list(N) == [0, 4, 5]
    assert list(steps.local_set(j0, j1, N)) == [2, 3, 0, 4, 5]
    assert steps.blocks(7, 3) == [(0, 3), (3, 6), (6, 7)]
    cand = {2: np.array([0, 2]), 3: np.array([3, 5])}
    freec = steps.screen(G_J, A_J, lam, j0, j1, cand)
    assert [list(f) for f in freec] == [[0, 2], [3, 5]]
    D = steps.delta_matrix(n, r, c, np.arange(1.0, 6.0))
    assert D[0, 2] == D[2, 0] == 1.0 and D[3, 4] == D[4, 3] == 4.0 and np.count_nonzero(D) == 8


def test_inverse_columns_residual():
    A, _, _, _ = _structured(12)
    cols = [1, 4, 7]
    W = steps.inverse_columns(A, cols)
    E = np.zeros((A.shape[0], 3)); E[cols, range(3)] = 1.0
    np.testing.assert_allclose(A @ W, E, atol=1e-12)


def test_level_candidates_hand_worked():
    n = 4
    ranking = np.array([0 * n + 0, 1 * n + 1, 0 * n + 3, 1 * n + 2, 2 * n + 2], dtype=np.int64)
    cand = steps.level_candidates(ranking, 4, n)
    assert [list(cand[c]) for c in range(n)] == [[0, 3], [1, 2], [1], [0]]


# ---------------------------------------------------------------- PCD-CG pins

def test_block_model_is_the_second_order_expansion_of_f():
    """q(Delta) - q(0) agrees with F(A + Delta) - F(A) up to O(|Delta|^3)
    (Section 5.1: the model is the second-order expansion of the smooth part
    plus the exact l1 term)."""
    from oracle import pcd
    A, _, _, _ = _structured(13, n=6, I=(0, 1), N=(4,))
    S = _structured(14, n=6, I=(0, 1), N=(4,))[0] / 3
    lam = 0.2
    W = np.linalg.inv(A)
    ri, ci = np.triu_indices(6)
    rng = np.random.default_rng(15)
    dir_ = rng.standard_normal(ri.size)
    errs = []
    for t in (1e-2, 5e-3, 2.5e-3):
        Dv = t * dir_
        Dm = steps.delta_matrix(6, ri, ci, Dv)
        q = pcd.block_model(W, ri, ci, S[ri, ci], A[ri, ci], lam, Dv) - \
            pcd.block_model(W, ri, ci, S[ri, ci], A[ri, ci], lam, 0 * Dv)
        ref = _mp_objective_change(A, Dm, S, lam, 1.0)
        errs.append(abs(q - ref))
    # third order: halving Delta divides the error by about 8
    assert errs[0] / errs[1] == pytest.approx(8.0, rel=0.1)
    assert errs[1] / errs[2] == pytest.approx(8.0, rel=0.1)


def test_hessian_product_is_the_derivative_of_the_inverse():
    """(W P W) is the derivative of -(A + tP)^{-1} at t = 0 (central difference)."""
    from oracle import pcd
    A, _, _, _ = _structured(16, n=6, I=(0, 1), N=(4,))
    W = np.linalg.inv(A)
    ri, ci = np.triu_indices(6)
    p = np.random.default_rng(17).standard_normal(ri.size)
    P = steps.delta_matrix(6, ri, ci, p)
    h = 1e-5
    fd = (np.linalg.inv(A - h * P) - np.linalg.inv(A + h * P)) / (2 * h)
    np.testing.assert_allclose(pcd.hessian_product(W, ri, ci, p), fd[ri, ci], atol=1e-8)


def test_pcd_cg_separable_model_is_solved_in_one_step():
    """With W diagonal the model separates by coordinate: the first PCD
    direction is every coordinate's exact minimiser (found here by 1-D
    brute-force minimisation) and the step 1 lies on the grid, so PCD-CG
    returns the exact solution."""
    from oracle import pcd
    nj = 5
    W = np.diag([1.5, 0.8, 1.2, 2.0, 0.6])
    rng = np.random.default_rng(18)
    S = rng.standard_normal((nj, nj)) * 0.5; S = S + S.T
    A = rng.standard_normal((nj, nj)) * 0.2; A = A + A.T
    lam = 0.3
    ri, ci = np.triu_indices(nj)
    Sv, Av = S[ri, ci], A[ri, ci]
    D, its, _ = pcd.pcd_cg(W, ri, ci, Sv, Av, lam, max_iter=10, tol=1e-12)
    for k in range(ri.size):
        def f(mu, k=k):
            e = np.zeros(ri.size); e[k] = mu
            return pcd.block_model(W, ri, ci, Sv, Av, lam, e)
        r = so.minimize_scalar(f, bracket=(-3, 3), tol=1e-14)
        best = min([r.x, -Av[k]], key=f)
        assert D[k] == pytest.approx(best, abs=1e-7)


def test_bruteforce_closed_forms():
    # n = 1: a = 1/(s + lam); n = 2 with |s12| > lam: W* = S + lam sign pattern
    assert bruteforce.solve(np.array([[1.7]]), 0.3)[0, 0] == pytest.approx(0.5, rel=1e-10)
    S = np.array([[1.3, 0.6], [0.6, 0.9]])
    lam = 0.2
    W = np.array([[1.3 + lam, 0.6 - lam], [0.6 - lam, 0.9 + lam]])
    np.testing.assert_allclose(bruteforce.solve(S, lam), np.linalg.inv(W), rtol=1e-9)


# ---------------------------------------------------------------- every oracle function is pinned

PINS = {
    "core.covariance": ["test_covariance_hand_worked_example",
                        "test_covariance_entries_by_loops_and_structure"],
    "core.cholesky_lower": ["test_logdet_pd_and_cholesky_closed_forms"],
    "core.logdet_pd": ["test_logdet_pd_and_cholesky_closed_forms",
                       "test_schur_line_matrices_match_direct_logdet"],
    "core.logdet_identity_plus": ["test_logdet_identity_plus_against_high_precision",
                                  "test_logdet_identity_plus_keeps_small_terms"],
    "core.inverse_pd": ["test_inverse_pd_is_an_inverse"],
    "core.objective": ["test_objective_closed_form_and_gradient_by_differences",
                       "test_diagonal_regime_closed_form"],
    "core.gradient": ["test_objective_closed_form_and_gradient_by_differences"],
    "core.min_norm_subgradient": ["test_min_norm_subgradient_by_brute_force"],
    "core.kkt_max": ["test_min_norm_subgradient_by_brute_force"],
    "core.kkt_l1": ["test_min_norm_subgradient_by_brute_force"],
    "core.free_mask": ["test_free_mask_and_support_pairs_hand_worked"],
    "core.support_pairs": ["test_free_mask_and_support_pairs_hand_worked"],
    "quic_plain.abs_change": ["test_abs_change_and_l1_change_exact_cases"],
    "quic_plain.objective_change": ["test_objective_change_against_high_precision",
                                    "test_objective_change_matches_difference"],
    "quic_plain.linesearch_dense": ["test_linesearch_skips_non_pd_trials"],
    "quic_plain.solve": ["test_diagonal_regime_closed_form", "test_lambda_zero_gives_inverse_covariance",
                         "test_one_variable", "test_two_variables_closed_form",
                         "test_bruteforce_support_enumeration", "test_kkt_certificate_and_diag_identity"],
    "quic_plain.solve_from_samples": ["test_kkt_certificate_and_diag_identity"],
    "steps.blocks": ["test_block_sets_hand_worked"],
    "steps.cov_block": ["test_covariance_hand_worked_example",
                        "test_cov_block_rows_by_loops_and_symmetric_diagonal_block"],
    "steps.inverse_columns": ["test_inverse_columns_residual"],
    "steps.screen": ["test_block_sets_hand_worked"],
    "steps.coordinates": ["test_block_sets_hand_worked"],
    "steps.neighborhood": ["test_block_sets_hand_worked"],
    "steps.local_set": ["test_block_sets_hand_worked"],
    "steps.cd_block": ["test_coarse_solution_correspondence", "test_block_updates_are_monotone"],
    "steps.delta_matrix": ["test_block_sets_hand_worked"],
    "steps.block_update": ["test_block_updates_are_monotone", "test_ml_bcd_matches_solution_oracle"],
    "steps.schur_line_matrices": ["test_schur_line_matrices_match_direct_logdet",
                                  "test_printed_b2_sign_would_be_wrong"],
    "steps.schur_logdet_change": ["test_schur_line_matrices_match_direct_logdet"],
    "steps.w_block_from_neighbors": ["test_neighbour_identity_app_a2"],
    "steps.hierarchy": ["test_hierarchy_sizes_and_order", "test_hierarchy_nested_and_terminates"],
    "steps.level_candidates": ["test_level_candidates_hand_worked",
                               "test_coarse_solution_correspondence"],
    "mlbcd.relax": ["test_block_updates_are_monotone", "test_coarse_solution_correspondence"],
    "mlbcd.supp_keys": ["test_ml_bcd_matches_solution_oracle"],
    "mlbcd.solve": ["test_ml_bcd_matches_solution_oracle", "test_bruteforce_support_enumeration",
                    "test_diagonal_regime_closed_form"],
    "pcd.block_model": ["test_block_model_is_the_second_order_expansion_of_f"],
    "pcd.l1_change": ["test_abs_change_and_l1_change_exact_cases"],
    "pcd.hessian_product": ["test_hessian_product_is_the_derivative_of_the_inverse"],
    "pcd.pcd_cg": ["test_pcd_cg_separable_model_is_solved_in_one_step",
                   "test_pcd_cg_converges_to_the_cd_minimiser",
                   "test_pcd_first_step_is_the_grid_minimiser_of_the_model"],
    "bruteforce.solve": ["test_bruteforce_closed_forms"],
    "cd.cd_sweeps": ["test_single_coordinate_step_is_1d_argmin", "test_cd_converges_to_model_kkt"],
}


def test_every_oracle_function_has_a_pin():
    """Every public function of the oracle is named above with the tests that
    pin it to something other than itself, and those tests exist here."""
    import inspect
    from oracle import bruteforce as m_bf, cd as m_cd, core as m_core, mlbcd as m_ml
    from oracle import pcd as m_pcd, quic_plain as m_q, steps as m_st
    mods = dict(core=m_core, quic_plain=m_q, steps=m_st, mlbcd=m_ml, pcd=m_pcd, bruteforce=m_bf,
                cd=m_cd)
    here = globals()
    for mname, mod in mods.items():
        for fname, fn in inspect.getmembers(mod, inspect.isfunction):
            if fn.__module__ != mod.__name__ or fname.startswith("_") or fname == "build":
                continue
            key = f"{mname}.{fname}"
            assert key in PINS, f"{key} has no pin"
    for key, tests in PINS.items():
        for t in tests:
            assert t in here and callable(here[t]), f"{key}: pin {t} is not a test here"
