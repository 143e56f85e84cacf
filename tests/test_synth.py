"""The seeded input generators: shapes, determinism, and exactness of the sampling solve."""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from synth import generators as g


def test_precision_shapes_and_dominance():
    P = g.chain_precision(50)
    assert P.nnz == 50 + 2 * 49
    assert np.allclose(P.diagonal(), 1.25)
    G = g.grid_precision(10, 10)
    assert G.shape == (100, 100)
    assert G.nnz == 100 + 2 * (2 * 10 * 9)
    rng = np.random.default_rng(0)
    R = g.random_precision(1000, 5000, rng)
    off = abs(R).sum(axis=1).A.ravel() - R.diagonal()
    assert np.all(R.diagonal() >= 1.1 * off - 1e-12)
    assert abs((R - R.T)).max() == 0
    vals = sp.triu(R, 1).data
    assert np.all((np.abs(vals) >= 0.05) & (np.abs(vals) <= 0.1))


def test_gram_split_reproduces_precision():
    rng = np.random.default_rng(1)
    P = g.random_precision(300, 1500, rng)
    G = g._split_gram_factor(P)
    assert abs(G @ G.T - P).max() < 1e-14


def test_sampling_solve_matches_direct_solve():
    rng = np.random.default_rng(2)
    P = g.random_precision(400, 2000, rng)
    Z = rng.standard_normal((400, 7))
    Y = g._chebyshev_solve(P, Z)
    Yd = spla.spsolve(P.tocsc(), Z)
    assert np.abs(Y - Yd).max() < 1e-11


def test_seeded_workload_is_deterministic():
    X1, P1, s1 = g.workload("chain_n64_m48")
    X2, P2, s2 = g.workload("chain_n64_m48")
    assert X1.shape == (48, 64) and X1.flags["C_CONTIGUOUS"]
    assert np.array_equal(X1, X2)


def test_sample_covariance_approaches_sigma():
    rng = np.random.default_rng(3)
    P = g.grid_precision(6, 6)
    X = g.sample_gaussian(P, 40000, rng)
    S = X.T @ X / X.shape[0]
    Sig = np.linalg.inv(P.toarray())
    assert np.abs(S - Sig).max() < 0.1


def test_request_stream_ranges():
    reqs = g.request_stream(64, seed=4, rate=10.0)
    assert len(reqs) == 64
    assert all(500 <= r["n"] <= 8000 and r["m"] == r["n"] // 2 for r in reqs)
    assert all(0.05 <= r["lam"] <= 0.5 for r in reqs)
    ts = [r["t"] for r in reqs]
    assert ts == sorted(ts) and ts[0] == 0.0


def test_delaunay_laplacian_is_a_dirichlet_graph_laplacian():
    """Section 8.1: -1 on every Delaunay edge, the degree on the diagonal, the
    points near the boundary deleted; positive definite, 6-7 non-zeros a row."""
    P = g.delaunay_precision(3000, np.random.default_rng(6))
    n = P.shape[0]
    assert 0.85 * 3000 < n < 3000
    assert abs(P - P.T).max() == 0
    off = sp.triu(P, 1).data
    assert np.all(off == -1.0)
    # the diagonal is the full graph's degree: at least the remaining off-diagonal count
    cnt = np.diff(P.indptr) - 1
    assert np.all(P.diagonal() >= cnt)
    assert 5.5 < P.nnz / n < 7.5
    lam_min = spla.eigsh(P.tocsc(), k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    assert lam_min > 0


def test_normalized_samples_have_unit_diagonal():
    X, P, spec = g.workload("delaunay_n700_m200")
    S_diag = np.mean(X * X, axis=0)
    assert np.allclose(S_diag, 1.0, atol=1e-12)
    assert np.allclose(X.mean(axis=0), 0.0, atol=1e-12)
    assert spec["n"] == X.shape[1] == P.shape[0]


def test_weakly_dominant_sampling_solve_is_exact():
    """The Laplacian's samples come from a sparse LU solve: P Y = G xi exactly."""
    rng = np.random.default_rng(7)
    P = g.delaunay_precision(1500, rng)
    assert not g._strictly_dominant(P)
    X = g.sample_gaussian(P, 40, np.random.default_rng(8))
    G = g._split_gram_factor(P)
    xi = np.random.default_rng(8).standard_normal((G.shape[1], 40))
    assert np.abs(P @ X.T - G @ xi).max() < 1e-9
