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
