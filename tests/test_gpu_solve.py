"""End-to-end parity of sic_solve against the CPU oracle (through the C-ABI).

Bar (float64 path): identical support, exact KKT max-norm of the GPU result
<= 1e-6 (measured by the oracle with a dense inverse), relative objective
within 1e-8 of the oracle's minimiser.
"""

import numpy as np
import pytest

from oracle import core, quic_plain
from synth import workload
from tests.helpers import announce, csr_to_dense, check_csr_valid

pytestmark = pytest.mark.gpu


def _solve(X, lam, tol, **opts):
    from paper_1607_00315_amd import sic
    with sic.Context(**opts) as c:
        (rp, col, val), info, trace = c.solve(X, lam, tol)
    n = X.shape[1]
    check_csr_valid(rp, col, val, n)
    return csr_to_dense(rp, col, val, n), info


def _exact_kkt(A, S, lam):
    W = np.linalg.inv(A)
    return core.kkt_max(S - W, A, lam)


@pytest.mark.parametrize("name,multilevel,cd_form", [
    ("chain_n200_m100", True, "hessian"), ("chain_n200_m100", False, "hessian"),
    ("chain_n200_m100", True, "u"), ("chain_n64_m48", True, "hessian"),
    ("random_n600_m300", True, "hessian"), ("random_n600_m300", True, "u"),
    ("grid_n900_m600", True, "hessian"), ("chain_n200_m100", True, "pcd"),
    ("random_n600_m300", True, "pcd"), ("grid_n900_m600", False, "pcd"),
    ("chain_n200_m100", True, "mixed"), ("random_n600_m300", True, "mixed"),
    ("grid_n900_m600", True, "mixed"), ("random_n600_m300", True, "mixed_formed"),
    ("grid_n900_m600", True, "mixed_formed")])
def test_solve_matches_oracle(name, multilevel, cd_form):
    from paper_1607_00315_amd import sic
    X, P, spec = workload(name)
    lam = spec["lam"]
    S = core.covariance(X)
    announce(f"solve {name} lam={lam} b={spec['block']} multilevel={multilevel} cd={cd_form}")
    flags = 0 if multilevel else sic.FLAG_NO_MULTILEVEL
    # mixed: float CG (and float coordinate Hessians) while far from the optimum,
    # then float64 cycles, S_J from the cached float64 columns; mixed_formed also
    # forms S_J in bfloat16 / float in those cycles (no cache). The bars below
    # are the float64 path's
    if cd_form == "mixed_formed":
        flags |= sic.FLAG_NO_S_CACHE
    A, info = _solve(X, lam, 1e-7, block=spec["block"], flags=flags,
                     cd_hessian_max=-1 if cd_form == "u" else 0,
                     pcd_min_coords=1 if cd_form == "pcd" else -1,
                     precision=sic.SIC_MIXED if cd_form.startswith("mixed") else sic.SIC_FP64)
    Aq, _ = quic_plain.solve(S, lam, tol=1e-12)
    assert np.array_equal(A, A.T)
    assert np.array_equal(A != 0, Aq != 0), \
        f"support differs: {np.count_nonzero(A)} vs {np.count_nonzero(Aq)}"
    assert _exact_kkt(A, S, lam) <= 1e-6
    F, Fq = core.objective(A, S, lam), core.objective(Aq, S, lam)
    assert abs(F - Fq) <= 1e-8 * abs(Fq)
    # the tracked objective sums line-search changes computed with CG-approximate
    # W (relative residual 1e-5 / 1e-4 in the first cycle), so it is an estimate:
    # its drift is bounded by the CG tolerance times the total step length
    assert abs(info["objective"] - F) <= 1e-6 * abs(F)
    assert info["status"] == 0


def test_diagonal_regime():
    X, P, spec = workload("chain_n64_m48")
    S = core.covariance(X)
    lam = 1.01 * np.max(np.abs(S - np.diag(np.diag(S))))
    announce("solve diagonal regime chain_n64")
    A, info = _solve(X, lam, 1e-9, block=16)
    np.testing.assert_allclose(A, np.diag(1.0 / (np.diag(S) + lam)), rtol=1e-12, atol=0)


def test_lambda_zero_many_samples():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((400, 40)) @ np.diag(np.linspace(0.5, 2.0, 40))
    S = core.covariance(X)
    announce("solve lambda=0 n=40 m=400")
    A, info = _solve(X, 0.0, 1e-9, block=16)
    np.testing.assert_allclose(A, np.linalg.inv(S), rtol=1e-7, atol=1e-9)


def test_single_variable_and_tiny_blocks():
    X = np.array([[1.0], [2.0], [-1.0]])
    announce("solve n=1")
    A, info = _solve(X, 0.3, 1e-12, block=8)
    assert A[0, 0] == pytest.approx(1.0 / (2.0 + 0.3), rel=1e-14)
    X, P, spec = workload("chain_n64_m48")
    S = core.covariance(X)
    announce("solve chain_n64 b=1 and b=7")
    Aq, _ = quic_plain.solve(S, spec["lam"], tol=1e-12)
    for b in (1, 7):
        A, info = _solve(X, spec["lam"], 1e-7, block=b)
        assert np.array_equal(A != 0, Aq != 0)


def test_invalid_arguments_rejected():
    from paper_1607_00315_amd import sic
    X = np.ones((5, 10))
    announce("invalid arguments")
    with sic.Context() as c:
        for lam, tol in [(-1.0, 1e-6), (0.1, 0.0), (0.0, 1e-6)]:   # lam=0 with m <= n
            with pytest.raises(sic.SicError) as e:
                c.solve(X, lam, tol)
            assert e.value.code == sic.SIC_EINVAL
        Xbad = np.ones((20, 4))
        Xbad[3, 2] = np.nan
        with pytest.raises(sic.SicError) as e:
            c.solve(Xbad, 0.1, 1e-6)
        assert e.value.code == sic.SIC_ENONFINITE


def test_device_input_pointer():
    import torch
    X, P, spec = workload("chain_n64_m48")
    announce("solve with a device pointer for X")
    A1, _ = _solve(X, spec["lam"], 1e-8, block=16)
    A2, _ = _solve(torch.from_numpy(X).cuda(), spec["lam"], 1e-8, block=16)
    assert np.array_equal(A1, A2)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_full_size_grid_solve(precision):
    """The benchmark workload (n = 10,000, m = 5,000, lambda = 0.08, block 256)
    at full size, in the benchmark's launch configuration:
      * support identical to the oracle's minimiser (stored by
        tests/golden/make_golden.py, which calls only oracle/);
      * objective within 1e-8 of the oracle's F*, evaluated exactly in float64;
      * a KKT certificate on 48 sampled columns: W columns by a sparse direct
        solve on the CPU, S columns from the samples, |g| <= lam off the
        support and g = -lam sign(A) on it, within 1e-6."""
    import json
    import os
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    from paper_1607_00315_amd import sic
    name = "grid_n10000_m5000"
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    golden = json.load(open(os.path.join(gdir, f"{name}.json")))
    gkeys = np.load(os.path.join(gdir, f"{name}_support.npz"))["keys"]
    X, P, spec = workload(name)
    lam, n, m = spec["lam"], X.shape[1], X.shape[0]
    announce(f"full-size solve {name} precision={precision}")
    prec = sic.SIC_MIXED if precision == "mixed" else sic.SIC_FP64
    with sic.Context(block=spec["block"], precision=prec) as c:
        (rp, col, val), info, _ = c.solve(X, lam, 1e-6)
    assert info["status"] == 0 and info["kkt_max"] <= 1e-6
    check_csr_valid(rp, col, val, n)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    keep = col >= rows
    keys = np.sort(rows[keep] * n + col[keep].astype(np.int64))
    assert np.array_equal(keys, gkeys), "support differs from the oracle's minimiser"
    A = sp.csr_matrix((val, col, rp), shape=(n, n))
    assert (abs(A - A.T) > 0).nnz == 0
    # exact objective: log det by a sparse Cholesky-free route (LU of the SPD
    # iterate), tr(SA) from the samples
    lu = spl.splu(A.tocsc())
    logdet = float(np.sum(np.log(np.abs(lu.U.diagonal()))))
    XA = (A @ X.T).T
    tr = float(np.sum(XA * X)) / m
    F = -logdet + tr + lam * float(np.abs(val).sum())
    assert abs(F - golden["F_star"]) <= 1e-8 * abs(golden["F_star"])
    # KKT certificate on sampled columns
    rng = np.random.default_rng(7)
    cols = np.sort(rng.choice(n, 48, replace=False))
    E = np.zeros((n, cols.size))
    E[cols, np.arange(cols.size)] = 1.0
    Wc = lu.solve(E)
    Sc = X.T @ X[:, cols] / m
    G = Sc - Wc
    Ac = A[:, cols].toarray()
    on = Ac != 0
    assert np.max(np.abs(G[on] + lam * np.sign(Ac[on]))) <= 1e-6
    assert np.max(np.abs(G[~on])) <= lam + 1e-6


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_repeat_solves_on_one_context_are_identical(precision):
    """A context keeps its workspace, its problem storage and the CG's
    first-check predictions between solves; none of that may change a result.
    One context solves A, then a smaller problem B, then (after a failed
    solve) A again; each result must equal, bit for bit, the same problem
    solved on a fresh context."""
    from paper_1607_00315_amd import sic
    prec = sic.SIC_MIXED if precision == "mixed" else sic.SIC_FP64
    XA, _, sa = workload("random_n600_m300")
    XB, _, sb = workload("chain_n200_m100")
    opts = dict(block=64, precision=prec)
    announce(f"repeat solves on one context ({precision})")

    def fresh(X, lam):
        with sic.Context(**opts) as c:
            return c.solve(X, lam, 1e-7)[0]

    bad = np.ones((20, 4))
    bad[3, 2] = np.nan
    with sic.Context(**opts) as c:
        a1 = c.solve(XA, sa["lam"], 1e-7)[0]
        b1 = c.solve(XB, sb["lam"], 1e-7)[0]
        with pytest.raises(sic.SicError):
            c.solve(bad, 0.1, 1e-6)
        a2 = c.solve(XA, sa["lam"], 1e-7)[0]
    a0, b0 = fresh(XA, sa["lam"]), fresh(XB, sb["lam"])
    for got, want in ((a1, a0), (a2, a0), (b1, b0)):
        for g, w in zip(got, want):
            assert np.array_equal(g, w)
