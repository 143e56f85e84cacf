"""Warm starts, lambda paths, failure codes and the convergence certificate,
through the C-ABI against the CPU oracle.

What is checked:
  * every result of a warm-started lambda path (solved as one batch problem
    and as one served request) against the oracle's minimiser at that lambda:
    identical support, objective within 1e-8 relative, exact KKT <= 1e-6;
  * a user warm start A0 (positive definite): the same bars, and the objective
    the library reports starts from F(A0) (Section 5, eq. (MLE_l1_prior));
  * a warm start with a positive diagonal that is not positive definite is
    refused with SIC_ENOTPD (the line search of Section 6.1.2 needs a PD start);
  * conjugate gradients stopped at cg_max_iter end the solve with SIC_ENOCONV
    and return the last accepted (positive definite) iterate;
  * the KKT value a converged solve reports is the exact one of its result;
  * submissions from one thread while another waits (the server's request
    table grows under the waiter).
"""

import threading

import numpy as np
import pytest

from oracle import core, quic_plain
from synth import workload
from tests.helpers import announce, check_csr_valid, csr_to_dense, dense_to_csr

pytestmark = pytest.mark.gpu

TOL = 1e-6
PATH = [0.4, 0.3, 0.2]


def _oracle(S, lam):
    A, _ = quic_plain.solve(S, lam, tol=1e-12)
    return A


def _check_against_oracle(A, Aq, S, lam, info=None):
    assert np.array_equal(A != 0, Aq != 0), \
        f"support differs: {np.count_nonzero(A)} vs {np.count_nonzero(Aq)}"
    W = np.linalg.inv(A)
    assert core.kkt_max(S - W, A, lam) <= TOL
    F, Fq = core.objective(A, S, lam), core.objective(Aq, S, lam)
    assert abs(F - Fq) <= 1e-8 * abs(Fq), (F, Fq)
    if info is not None:
        assert np.isfinite(info["objective"])
        assert abs(info["objective"] - F) <= 1e-6 * abs(F)


@pytest.fixture(scope="module")
def rnd600():
    X, P, spec = workload("random_n600_m300")
    S = core.covariance(X)
    return X, S, spec, {lam: _oracle(S, lam) for lam in PATH}


def test_lambda_path_batch_matches_oracle(rnd600):
    from paper_1607_00315_amd import sic
    X, S, spec, ref = rnd600
    announce(f"lambda path {PATH} random_n600_m300 as one batch problem vs the oracle")
    with sic.Context(block=spec["block"]) as c:
        code, res = c.solve_batch([dict(X=X, lambda_path=PATH, tol=TOL)])
    assert code == 0
    n = X.shape[1]
    for lam, ((rp, col, val), info) in zip(PATH, res):
        check_csr_valid(rp, col, val, n)
        assert info["status"] == 0
        _check_against_oracle(csr_to_dense(rp, col, val, n), ref[lam], S, lam, info)


def test_lambda_path_served_matches_oracle(rnd600):
    from paper_1607_00315_amd import sic
    X, S, spec, ref = rnd600
    announce(f"lambda path {PATH} random_n600_m300 as one served request vs the oracle")
    with sic.Server(slots=2, block=spec["block"]) as srv:
        t = srv.submit(dict(X=X, lambda_path=PATH, tol=TOL))
        code, results, infos, _ = srv.wait(t, timeout=300.0)
    assert code == 0
    n = X.shape[1]
    for lam, A, info in zip(PATH, results, infos):
        _check_against_oracle(csr_to_dense(*A, n), ref[lam], S, lam, info)


def test_warm_start_matches_oracle(rnd600):
    from paper_1607_00315_amd import sic
    X, S, spec, ref = rnd600
    n = X.shape[1]
    announce("warm start from the oracle's minimiser at lambda 0.3, solved at 0.2")
    A0 = ref[0.3]
    with sic.Context(block=spec["block"]) as c:
        code, res = c.solve_batch([dict(X=X, lam=0.2, tol=TOL, A0=dense_to_csr(A0))])
    assert code == 0
    (rp, col, val), info = res[0]
    _check_against_oracle(csr_to_dense(rp, col, val, n), ref[0.2], S, 0.2, info)
    announce("warm start at the minimiser itself: the reported objective is F(A0)")
    with sic.Context(block=spec["block"]) as c:
        code, res = c.solve_batch([dict(X=X, lam=0.2, tol=TOL, A0=dense_to_csr(ref[0.2]))])
    assert code == 0
    Fq = core.objective(ref[0.2], S, 0.2)
    assert abs(res[0][1]["objective"] - Fq) <= 1e-9 * abs(Fq)
    # the first cycle's CG runs at the paper's tolerances (1e-5 / 1e-4), so its
    # KKT measure may need one tightened cycle to certify 1e-6
    assert res[0][1]["cycles"] <= 2
    (rp, col, val), info = res[0]
    _check_against_oracle(csr_to_dense(rp, col, val, n), ref[0.2], S, 0.2, info)


def test_non_pd_warm_start_is_refused():
    from paper_1607_00315_amd import sic
    X, P, spec = workload("chain_n64_m48")
    n = X.shape[1]
    # tridiagonal, diagonal 1 and off-diagonal 0.9: positive diagonal, eigenvalues
    # 1 + 1.8 cos(k pi / (n + 1)) reach -0.8
    A0 = np.eye(n) + 0.9 * (np.eye(n, k=1) + np.eye(n, k=-1))
    assert np.linalg.eigvalsh(A0).min() < 0
    announce("non-PD warm start with a positive diagonal (chain_n64_m48)")
    with sic.Context(block=spec["block"]) as c:
        code, res = c.solve_batch([dict(X=X, lam=spec["lam"], tol=TOL, A0=dense_to_csr(A0))])
        assert code == sic.SIC_ENOTPD, code
        assert res[0][1]["status"] == sic.SIC_ENOTPD
        # the context stays usable: a PD warm start next
        A1 = np.eye(n) + 0.3 * (np.eye(n, k=1) + np.eye(n, k=-1))
        code, res = c.solve_batch([dict(X=X, lam=spec["lam"], tol=TOL, A0=dense_to_csr(A1))])
        assert code == 0


def test_cg_iteration_cap_gives_enoconv():
    from paper_1607_00315_amd import sic
    X, P, spec = workload("random_n600_m300")
    n = X.shape[1]
    announce("cg_max_iter = 1 on random_n600_m300: SIC_ENOCONV with the last accepted iterate")
    with sic.Context(block=spec["block"], cg_max_iter=1) as c:
        (rp, col, val), info, _ = c.solve(X, spec["lam"], TOL)
        assert info["status"] == sic.SIC_ENOCONV
        check_csr_valid(rp, col, val, n)
        A = csr_to_dense(rp, col, val, n)
        assert np.linalg.eigvalsh(A).min() > 0
    # the same context after the failure: a normal solve still matches the oracle
    S = core.covariance(X)
    with sic.Context(block=spec["block"]) as c:
        (rp, col, val), info, _ = c.solve(X, spec["lam"], TOL)
    assert info["status"] == 0
    _check_against_oracle(csr_to_dense(rp, col, val, n), _oracle(S, spec["lam"]), S, spec["lam"])


def test_reported_kkt_is_the_exact_one():
    from paper_1607_00315_amd import sic
    X, P, spec = workload("chain_n200_m100")
    n = X.shape[1]
    S = core.covariance(X)
    announce("chain_n200_m100 to KKT 1e-7: the reported measure is the result's exact KKT")
    with sic.Context(block=spec["block"]) as c:
        (rp, col, val), info, _ = c.solve(X, spec["lam"], 1e-7)
    assert info["status"] == 0
    A = csr_to_dense(rp, col, val, n)
    exact = core.kkt_max(S - np.linalg.inv(A), A, spec["lam"])
    assert info["kkt_max"] <= 1e-7
    assert abs(info["kkt_max"] - exact) <= 1e-9


def test_submit_while_another_thread_waits():
    from paper_1607_00315_amd import sic
    from tests.test_gpu_serve import _mix
    probs = _mix(count=12, seed=27, n_lo=200, n_hi=500)
    announce("12 submissions from one thread while another waits on the first")
    errors, got = [], {}
    with sic.Server(slots=2) as srv:
        first = srv.submit(probs[0])

        def waiter():
            try:
                got["first"] = srv.wait(first, timeout=300.0)
            except Exception as e:   # noqa: BLE001
                errors.append(e)

        th = threading.Thread(target=waiter)
        th.start()
        tickets = [srv.submit(p) for p in probs[1:]]
        th.join()
        rest = [srv.wait(t, timeout=300.0) for t in tickets]
    assert not errors, errors
    assert got["first"][0] == 0
    assert all(r[0] == 0 for r in rest)


@pytest.mark.parametrize("name,multilevel", [("random_n600_m300", False),
                                             ("delaunay_n700_m200", True)])
def test_continuation_matches_oracle(name, multilevel):
    """The continuation schedule of Section 8 (BCDcont without the levels):
    three cycles at larger lambdas, then lambda; the result is the oracle's
    minimiser at lambda, and the reported objective is F at lambda."""
    from paper_1607_00315_amd import sic
    X, P, spec = workload(name)
    n = X.shape[1]
    lam = spec["lam"]
    S = core.covariance(X)
    flags = sic.FLAG_CONTINUATION | (0 if multilevel else sic.FLAG_NO_MULTILEVEL)
    announce(f"continuation {name} lam={lam} multilevel={multilevel}")
    with sic.Context(block=spec["block"], flags=flags, trace_cap=64) as c:
        (rp, col, val), info, trace = c.solve(X, lam, TOL)
    assert info["status"] == 0
    assert info["cycles"] >= 4
    _check_against_oracle(csr_to_dense(rp, col, val, n), _oracle(S, lam), S, lam, info)


@pytest.mark.parametrize("name", ["random_n600_m300", "delaunay_n700_m200"])
def test_warm_started_cg_matches_cold(name):
    """Warm starts of the block CG (each column of W_J started from the last
    inverse column computed for it) change only where the iterations begin:
    with and without them the result is the oracle's minimiser, and the warm
    run needs no more CG iterations than the cold one."""
    from paper_1607_00315_amd import sic
    X, P, spec = workload(name)
    n = X.shape[1]
    lam = spec["lam"]
    S = core.covariance(X)
    ref = _oracle(S, lam)
    its = {}
    for warm in (True, False):
        flags = 0 if warm else sic.FLAG_NO_WARM_CG
        announce(f"warm-start CG {name} lam={lam} warm={warm}")
        with sic.Context(block=spec["block"], flags=flags) as c:
            (rp, col, val), info, _ = c.solve(X, lam, TOL)
        assert info["status"] == 0
        _check_against_oracle(csr_to_dense(rp, col, val, n), ref, S, lam, info)
        its[warm] = info["cg_iterations"]
    assert its[True] <= its[False], its


def test_cached_s_columns_change_nothing():
    """Columns of S formed in one cycle are copied out in the next instead of
    formed again: the solve is bit for bit the one that forms every block."""
    from paper_1607_00315_amd import sic
    X, P, spec = workload("grid_n900_m600")
    lam = spec["lam"]
    out = {}
    for flags in (0, sic.FLAG_NO_S_CACHE):
        announce(f"cached S columns grid_n900_m600 flags={flags}")
        with sic.Context(block=spec["block"], flags=flags) as c:
            (rp, col, val), info, _ = c.solve(X, lam, 1e-8)
        assert info["status"] == 0 and info["cycles"] >= 2
        out[flags] = (rp, col, val, info["objective"])
    a, b = out[0], out[sic.FLAG_NO_S_CACHE]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2]) and a[3] == b[3]
