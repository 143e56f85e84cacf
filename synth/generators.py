"""Seeded sparse precision matrices and Gaussian samples.

Every generator takes an explicit ``numpy.random.Generator`` (PCG64 through
``numpy.random.default_rng(seed)``) so that the same seed gives the same bytes
on any machine with this numpy.

Sampling recipe (exact in law, no factorisation of P):
  * split the diagonally dominant precision P as G G^T: every stored
    off-diagonal pair (i, j) contributes the column sqrt|p_ij| (e_i + sign(p_ij) e_j)
    and every row the column sqrt(p_ii - sum_j |p_ij|) e_i;
  * z = G xi with xi ~ N(0, I) has covariance P;
  * y = P^{-1} z then has covariance P^{-1} P P^{-1} = P^{-1} = Sigma.
The linear solve P y = z is done by Chebyshev semi-iteration on the
Jacobi-scaled system, whose spectrum lies in [1 - rho, 1 + rho] with
rho = max_i sum_{j != i} |p_ij| / p_ii < 1 by diagonal dominance
(Gershgorin); see Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
Algorithm 12.1.  Matrices that are only weakly dominant (the planar graph
Laplacians, whose interior rows have p_ii equal to their off-diagonal sum) are
solved by a sparse LU factorisation instead.  Samples are returned as the
m x n matrix X whose rows are the draws (row-major float64), the layout the
solver consumes.

The planar-graph workloads follow Section 8.1 of the paper: n uniform points
in the unit square, edges of their Delaunay triangulation, precision -1 on
every edge and the vertex degree on the diagonal (a graph Laplacian, PSD with
the constant vector as null space), made definite by deleting the points
within 1/sqrt(n) of the square's boundary (the rows and columns of the rest
form a Dirichlet Laplacian).  Their samples are normalised as the paper's are:
each variable centred and scaled so that diag(X^T X / m) = 1.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# --------------------------------------------------------------------------
# precision matrices
# --------------------------------------------------------------------------

def chain_precision(n: int, diag: float = 1.25, off: float = -0.5) -> sp.csr_matrix:
    """Tridiagonal precision: P_ii = diag, P_{i,i+1} = P_{i+1,i} = off."""
    if n < 1:
        raise ValueError("n must be >= 1")
    main = np.full(n, diag, dtype=np.float64)
    side = np.full(max(n - 1, 0), off, dtype=np.float64)
    return sp.diags([side, main, side], [-1, 0, 1], shape=(n, n), format="csr")


def grid_precision(rows: int, cols: int, n: int | None = None,
                   diag: float = 1.0, off: float = -0.2) -> sp.csr_matrix:
    """4-neighbour grid precision on a rows x cols lattice, node r*cols + c.

    With ``n`` smaller than rows*cols the lattice is truncated to its first
    ``n`` nodes (row-major), which keeps every row diagonally dominant.
    """
    total = rows * cols
    if n is None:
        n = total
    if not (1 <= n <= total):
        raise ValueError("n must lie in [1, rows*cols]")
    ii, jj = [], []
    for node in range(n):
        r, c = divmod(node, cols)
        if c + 1 < cols and node + 1 < n:
            ii.append(node)
            jj.append(node + 1)
        if r + 1 < rows and node + cols < n:
            ii.append(node)
            jj.append(node + cols)
    ii = np.asarray(ii, dtype=np.int64)
    jj = np.asarray(jj, dtype=np.int64)
    vals = np.full(ii.size, off, dtype=np.float64)
    upper = sp.coo_matrix((vals, (ii, jj)), shape=(n, n))
    P = (upper + upper.T).tocsr()
    P = P + sp.diags(np.full(n, diag), 0, shape=(n, n), format="csr")
    return P.tocsr()


def random_precision(n: int, pairs: int, rng: np.random.Generator,
                     lo: float = 0.05, hi: float = 0.1,
                     diag_factor: float = 1.1) -> sp.csr_matrix:
    """Random sparse SPD precision.

    ``pairs`` index pairs (i, j), i != j, are drawn uniformly and deduplicated
    as unordered pairs; each gets a value of magnitude U[lo, hi] and a fair
    random sign. The diagonal is diag_factor times the row's absolute
    off-diagonal sum, or 1.0 for a row with no off-diagonal entry.
    """
    if n < 2:
        raise ValueError("n must be >= 2")
    i = rng.integers(0, n, size=pairs, dtype=np.int64)
    j = rng.integers(0, n - 1, size=pairs, dtype=np.int64)
    j = j + (j >= i)                       # uniform over j != i
    a = np.minimum(i, j)
    b = np.maximum(i, j)
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    mag = rng.uniform(lo, hi, size=key.size)
    sign = np.where(rng.integers(0, 2, size=key.size) == 1, 1.0, -1.0)
    vals = mag * sign
    upper = sp.coo_matrix((vals, (a, b)), shape=(n, n))
    P = (upper + upper.T).tocsr()
    absrow = np.asarray(abs(P).sum(axis=1)).ravel()
    d = np.where(absrow > 0, diag_factor * absrow, 1.0)
    P = P + sp.diags(d, 0, shape=(n, n), format="csr")
    return P.tocsr()


def delaunay_precision(points: int, rng: np.random.Generator) -> sp.csr_matrix:
    """Dirichlet graph Laplacian of a random planar (Delaunay) graph.

    ``points`` uniform points in the unit square; P_ij = -1 for every edge of
    their Delaunay triangulation, P_ii = the vertex degree; then the rows and
    columns of the points with a coordinate closer than 1/sqrt(points) to the
    boundary are deleted. The points keep their (random) drawing order, so the
    natural order of the variables has no locality.
    """
    from scipy.spatial import Delaunay
    if points < 16:
        raise ValueError("need at least 16 points")
    xy = rng.random((points, 2))
    tri = Delaunay(xy).simplices.astype(np.int64)
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [0, 2]]])
    e.sort(axis=1)
    key = np.unique(e[:, 0] * points + e[:, 1])
    a, b = key // points, key % points
    adj = sp.coo_matrix((np.ones(a.size), (a, b)), shape=(points, points))
    adj = (adj + adj.T).tocsr()
    deg = np.asarray(adj.sum(axis=1)).ravel()
    L = (sp.diags(deg) - adj).tocsr()
    h = 1.0 / math.sqrt(points)
    keep = np.nonzero(np.all((xy > h) & (xy < 1.0 - h), axis=1))[0]
    P = L[keep][:, keep].tocsr()
    P.sort_indices()
    return P


# --------------------------------------------------------------------------
# sampling
# --------------------------------------------------------------------------

def _split_gram_factor(P: sp.csr_matrix) -> sp.csr_matrix:
    """Sparse G with G G^T = P for a symmetric weakly diagonally dominant P."""
    n = P.shape[0]
    coo = sp.triu(P, k=1).tocoo()
    e = coo.nnz
    s = np.sqrt(np.abs(coo.data))
    rows = np.concatenate([coo.row, coo.col])
    cols = np.concatenate([np.arange(e), np.arange(e)])
    vals = np.concatenate([s, s * np.sign(coo.data)])
    d = P.diagonal() - (np.asarray(abs(P).sum(axis=1)).ravel() - np.abs(P.diagonal()))
    if np.any(d < -1e-12 * np.abs(P.diagonal())):
        raise ValueError("precision matrix is not diagonally dominant")
    d = np.sqrt(np.maximum(d, 0.0))
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([cols, e + np.arange(n)])
    vals = np.concatenate([vals, d])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, e + n))


def _chebyshev_solve(P: sp.csr_matrix, Z: np.ndarray, rtol: float = 1e-14,
                     max_iter: int = 5000) -> np.ndarray:
    """Solve P Y = Z (many right-hand sides) by Chebyshev semi-iteration.

    Works on the symmetrically Jacobi-scaled matrix D^{-1/2} P D^{-1/2},
    whose eigenvalues lie in [1 - rho, 1 + rho] (Gershgorin on D^{-1} P).
    """
    dg = P.diagonal().astype(np.float64)
    if np.any(dg <= 0):
        raise ValueError("precision diagonal must be positive")
    off = np.asarray(abs(P).sum(axis=1)).ravel() - np.abs(dg)
    rho = float(np.max(off / dg))
    if not rho < 1.0:
        raise ValueError("Jacobi-scaled spectrum bound needs strict dominance")
    s = 1.0 / np.sqrt(dg)
    Ps = sp.diags(s) @ P @ sp.diags(s)
    Ps = Ps.tocsr()
    B = Z * s[:, None]
    lo, hi = 1.0 - rho, 1.0 + rho
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    x = np.zeros_like(B)
    r = B.copy()
    bnorm = np.maximum(np.linalg.norm(B, axis=0), 1e-300)
    rho_k = 1.0 / sigma
    d = r / theta
    for it in range(max_iter):
        x += d
        r -= Ps @ d
        if it % 8 == 7:
            rel = np.max(np.linalg.norm(r, axis=0) / bnorm)
            if rel <= rtol:
                break
        rho_next = 1.0 / (2.0 * sigma - rho_k)
        d *= rho_next * rho_k
        d += (2.0 * rho_next / delta) * r
        rho_k = rho_next
    else:
        raise RuntimeError("Chebyshev sampling solve did not converge")
    return x * s[:, None]


def _strictly_dominant(P: sp.csr_matrix) -> bool:
    dg = np.abs(P.diagonal())
    off = np.asarray(abs(P).sum(axis=1)).ravel() - dg
    return bool(np.all(off < dg))


def sample_gaussian(P: sp.csr_matrix, m: int, rng: np.random.Generator) -> np.ndarray:
    """Draw m samples of N(0, P^{-1}); returns X (m x n, C-contiguous float64)."""
    P = sp.csr_matrix(P, dtype=np.float64)
    G = _split_gram_factor(P)
    xi = rng.standard_normal((G.shape[1], m))
    Z = G @ xi
    del xi
    if _strictly_dominant(P):
        Y = _chebyshev_solve(P, Z)
    else:
        Y = spla.splu(P.tocsc(), permc_spec="COLAMD").solve(np.asarray(Z))
    return np.ascontiguousarray(Y.T)


def normalize_samples(X: np.ndarray) -> np.ndarray:
    """Centre every variable and scale it so that diag(X^T X / m) = 1 (the
    normalisation of the paper's experiments, Section 8)."""
    X = X - X.mean(axis=0, keepdims=True)
    s = np.sqrt(np.mean(X * X, axis=0))
    s[s == 0] = 1.0
    return np.ascontiguousarray(X / s)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def _grid_dims(n: int) -> tuple[int, int]:
    r = int(math.isqrt(n))
    c = -(-n // r)
    return r, c


def _precision(kind: str, n: int, rng: np.random.Generator, random_pairs_per_node: int):
    if kind == "chain":
        return chain_precision(n)
    if kind == "grid":
        r, c = _grid_dims(n)
        return grid_precision(r, c, n=n)
    if kind == "random":
        return random_precision(n, random_pairs_per_node * n, rng)
    if kind == "delaunay":
        return delaunay_precision(n, rng)
    raise ValueError(f"unknown graph kind {kind!r}")


def _lambda_path(k: int = 8, hi: float = 0.5, lo: float = 0.05) -> list[float]:
    return [hi * (lo / hi) ** (i / (k - 1)) for i in range(k)]


# name -> (graph kind, n, m, seed, lambda (or path), block, random pairs per node)
WORKLOADS = {
    "chain_n200_m100": dict(kind="chain", n=200, m=100, seed=1, lam=0.1, block=32),
    "grid_n10000_m5000": dict(kind="grid", n=10000, m=5000, seed=2, lam=0.08, block=256,
                              grid=(100, 100)),
    "random_n100000_m200": dict(kind="random", n=100000, m=200, seed=3, lam=0.5, block=256,
                                pairs_per_node=5),
    "random_n20000_m1000_path": dict(kind="random", n=20000, m=1000, seed=5,
                                     lam=_lambda_path(), block=256, pairs_per_node=4),
    # small shapes of the same families, for tests that must finish in seconds
    "chain_n64_m48": dict(kind="chain", n=64, m=48, seed=11, lam=0.12, block=16),
    "grid_n400_m300": dict(kind="grid", n=400, m=300, seed=12, lam=0.1, block=64,
                           grid=(20, 20)),
    "grid_n900_m600": dict(kind="grid", n=900, m=600, seed=14, lam=0.08, block=128,
                           grid=(30, 30)),
    "random_n600_m300": dict(kind="random", n=600, m=300, seed=13, lam=0.2, block=128,
                             pairs_per_node=5),
    "grid_n2500_m1500": dict(kind="grid", n=2500, m=1500, seed=15, lam=0.08, block=256,
                             grid=(50, 50)),
    # Section 8.1 shapes: random planar graph Laplacians (n = the points drawn;
    # about 1% of them, those near the boundary, are deleted), normalised samples
    "delaunay_n125000_m200": dict(kind="delaunay", n=125000, m=200, seed=21, lam=0.7,
                                  block=256, normalize=True),
    "delaunay_n20000_m200": dict(kind="delaunay", n=20000, m=200, seed=22, lam=0.6,
                                 block=256, normalize=True),
    "delaunay_n700_m200": dict(kind="delaunay", n=700, m=200, seed=23, lam=0.5, block=64,
                               normalize=True),
    # Section 8.2 shapes (gene-expression data, n >> m): the datasets are not
    # available; planar-graph Gaussian samples of the same n and m, normalised
    # the same way, stand in for them
    "geo_n22283_m278": dict(kind="delaunay", n=22283, m=278, seed=24, lam=0.7, block=256,
                            normalize=True),
}


def workload(name: str):
    """Return (X, P, spec) for a named workload; X is m x n float64 row-major."""
    spec = dict(WORKLOADS[name])
    rng = np.random.default_rng(spec["seed"])
    n = spec["n"]
    if spec["kind"] == "grid" and "grid" in spec:
        P = grid_precision(*spec["grid"], n=n)
    else:
        P = _precision(spec["kind"], n, rng, spec.get("pairs_per_node", 5))
    X = sample_gaussian(P, spec["m"], rng)
    if spec.get("normalize"):
        X = normalize_samples(X)
    spec["points"] = n
    spec["n"] = X.shape[1]
    spec["name"] = name
    return X, P, spec


def request_stream(count: int = 256, seed: int = 4, rate: float = 1.0,
                   n_lo: int = 500, n_hi: int = 8000,
                   lam_lo: float = 0.05, lam_hi: float = 0.5):
    """Serving workload: Poisson arrivals of estimation problems.

    Returns a list of dicts with arrival time (seconds, at ``rate`` requests
    per second), graph kind, n, m = n // 2, lambda and the per-request seed;
    the samples themselves are drawn lazily by :func:`request_samples`.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    kinds = ["chain", "grid", "random"]
    out = []
    for k in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        out.append(dict(t=float(t[k]), kind=kinds[int(rng.integers(0, 3))], n=n, m=n // 2,
                        lam=float(rng.uniform(lam_lo, lam_hi)),
                        seed=int(rng.integers(0, 2**31 - 1)), block=256))
    return out


def request_samples(req: dict):
    rng = np.random.default_rng(req["seed"])
    P = _precision(req["kind"], req["n"], rng, 3)
    return sample_gaussian(P, req["m"], rng), P
