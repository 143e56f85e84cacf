"""Clustered blocks (SIC_FLAG_CLUSTER, Section 6.1) end to end through the
C-ABI, against the CPU oracle's minimiser: the relabelling only changes which
variables share a block, so the unique minimiser is the same. Bars as in
test_gpu_solve: identical support, exact KKT <= 1e-6, objective within 1e-8.
Also a warm-started lambda path with clustering (the problem stays relabelled
between lambdas; every result comes back in the caller's labels)."""

import numpy as np
import pytest

from oracle import core, quic_plain
from synth import workload
from tests.helpers import announce, check_csr_valid, csr_to_dense

pytestmark = pytest.mark.gpu


def _check(A, S, lam):
    Aq, _ = quic_plain.solve(S, lam, tol=1e-12)
    assert np.array_equal(A, A.T)
    assert np.array_equal(A != 0, Aq != 0), \
        f"support differs: {np.count_nonzero(A)} vs {np.count_nonzero(Aq)}"
    assert core.kkt_max(S - np.linalg.inv(A), A, lam) <= 1e-6
    F, Fq = core.objective(A, S, lam), core.objective(Aq, S, lam)
    assert abs(F - Fq) <= 1e-8 * abs(Fq)


@pytest.mark.parametrize("name,precision", [("delaunay_n700_m200", "f64"),
                                            ("grid_n900_m600", "f64"),
                                            ("random_n600_m300", "mixed")])
def test_clustered_solve_matches_oracle(name, precision):
    from paper_1607_00315_amd import sic
    X, P, spec = workload(name)
    lam = spec["lam"]
    n = X.shape[1]
    announce(f"clustered solve {name} lam={lam} b={spec['block']} {precision}")
    prec = sic.SIC_MIXED if precision == "mixed" else sic.SIC_FP64
    with sic.Context(block=spec["block"], flags=sic.FLAG_CLUSTER, precision=prec) as c:
        (rp, col, val), info, _ = c.solve(X, lam, 1e-7)
    assert info["status"] == 0
    check_csr_valid(rp, col, val, n)
    _check(csr_to_dense(rp, col, val, n), core.covariance(X), lam)


def test_clustered_lambda_path_matches_oracle():
    from paper_1607_00315_amd import sic
    X, P, spec = workload("delaunay_n700_m200")
    n = X.shape[1]
    S = core.covariance(X)
    path = [0.6, 0.5, 0.4]
    announce(f"clustered lambda path {path} delaunay_n700_m200")
    with sic.Context(block=spec["block"], flags=sic.FLAG_CLUSTER) as c:
        code, res = c.solve_batch([dict(X=X, lambda_path=path, tol=1e-7)])
    assert code == 0
    for lam, ((rp, col, val), info) in zip(path, res):
        check_csr_valid(rp, col, val, n)
        _check(csr_to_dense(rp, col, val, n), S, lam)
