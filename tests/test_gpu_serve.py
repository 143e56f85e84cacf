"""Serving loop (include/sic_serve.h) through the C-ABI.

What is checked:
  * every result served in a mix of concurrent problems is the one the same
    problem gives alone (sic_solve_batch on its own context): identical
    support, values and objective within 1e-12 relative (the kernels have no
    atomics, so the expected difference is zero);
  * served results match the oracle's minimiser on a case it solves quickly;
  * admission by device-memory footprint: with a budget that holds one
    problem at a time, no two requests run together; a problem larger than the
    budget is refused at submission;
  * a queued request can be cancelled; a lambda path is one request;
  * with several slots, requests do run at the same time.
"""

import numpy as np
import pytest

from oracle import core, quic_plain
from synth import workload
from synth.generators import request_samples, request_stream
from tests.helpers import announce, check_csr_valid, csr_to_dense

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _mix(count=10, seed=21, n_lo=200, n_hi=1100):
    reqs = request_stream(count, seed=seed, rate=1.0, n_lo=n_lo, n_hi=n_hi)
    out = []
    for r in reqs:
        X, _ = request_samples(r)
        out.append(dict(X=X, lam=r["lam"], tol=TOL, kind=r["kind"], n=r["n"]))
    return out


def _alone(p):
    from paper_1607_00315_amd import sic
    with sic.Context() as c:
        code, res = c.solve_batch([dict(X=p["X"], lam=p["lam"], tol=p["tol"])])
    return code, res[0]


def _same(a, b, n):
    (rp1, c1, v1), (rp2, c2, v2) = a, b
    assert np.array_equal(rp1, rp2) and np.array_equal(c1, c2), "support differs"
    scale = max(1.0, float(np.max(np.abs(v1))))
    assert np.max(np.abs(v1 - v2)) <= 1e-12 * scale


def test_served_mix_equals_alone():
    from paper_1607_00315_amd import sic
    probs = _mix()
    announce(f"serve mix of {len(probs)} problems, n in "
             f"[{min(p['n'] for p in probs)}, {max(p['n'] for p in probs)}], 4 slots")
    with sic.Server(slots=4) as srv:
        tickets = [srv.submit(p) for p in probs]
        served = [srv.wait(t, timeout=300.0) for t in tickets]
    announce("the same problems alone")
    for p, s in zip(probs, served):
        assert s is not None, "request timed out"
        code, results, infos, times = s
        alone_code, (alone_A, alone_info) = _alone(p)
        assert code == alone_code == 0, (code, alone_code)
        check_csr_valid(*results[0], p["n"])
        _same(results[0], alone_A, p["n"])
        F1, F2 = infos[0]["objective"], alone_info["objective"]
        assert abs(F1 - F2) <= 1e-12 * abs(F2)
        assert infos[0]["cycles"] == alone_info["cycles"]
        assert times["submitted"] <= times["admitted"] <= times["finished"]
    # concurrency: with 4 slots and 10 queued problems some intervals overlap
    iv = sorted((s[3]["admitted"], s[3]["finished"]) for s in served)
    overlap = any(iv[k + 1][0] < iv[k][1] for k in range(len(iv) - 1))
    assert overlap, "no two requests ran at the same time"
    assert len({s[3]["slot"] for s in served}) > 1


def test_served_result_matches_oracle():
    from paper_1607_00315_amd import sic
    X, P, spec = workload("chain_n200_m100")
    lam = spec["lam"]
    others = _mix(count=4, seed=22, n_lo=300, n_hi=800)
    announce("serve chain_n200_m100 among 4 others, compare with the oracle")
    with sic.Server(slots=3, block=spec["block"]) as srv:
        tk = [srv.submit(p) for p in others[:2]]
        t = srv.submit(dict(X=X, lam=lam, tol=1e-7))
        tk += [srv.submit(p) for p in others[2:]]
        code, results, infos, _ = srv.wait(t, timeout=300.0)
        for x in tk:
            assert srv.wait(x, timeout=300.0)[0] == 0
    assert code == 0
    n = X.shape[1]
    A = csr_to_dense(*results[0], n)
    S = core.covariance(X)
    Aq, _ = quic_plain.solve(S, lam, tol=1e-12)
    assert np.array_equal(A != 0, Aq != 0)
    assert core.kkt_max(S - np.linalg.inv(A), A, lam) <= 1e-6
    F, Fq = core.objective(A, S, lam), core.objective(Aq, S, lam)
    assert abs(F - Fq) <= 1e-8 * abs(Fq)


def test_admission_by_footprint_serialises_and_refuses():
    from paper_1607_00315_amd import sic
    probs = _mix(count=4, seed=23, n_lo=400, n_hi=700)
    with sic.Server(slots=4) as probe:
        fps = [probe.footprint(p) for p in probs]
    budget = int(1.5 * max(fps))       # room for one problem, never two
    assert all(2 * f > budget for f in fps)
    announce(f"serve 4 problems under a budget of {budget} bytes (footprints {fps})")
    with sic.Server(slots=4, hbm_budget=budget) as srv:
        big = _mix(count=1, seed=24, n_lo=3000, n_hi=3000)[0]
        assert srv.footprint(big) > budget
        with pytest.raises(sic.SicError) as e:
            srv.submit(big)
        assert e.value.code == sic.SIC_ENOMEM
        tickets = [srv.submit(p) for p in probs]
        served = [srv.wait(t, timeout=300.0) for t in tickets]
        st = srv.status()
    assert all(s[0] == 0 for s in served)
    iv = sorted((s[3]["admitted"], s[3]["finished"]) for s in served)
    assert all(iv[k + 1][0] >= iv[k][1] for k in range(len(iv) - 1)), \
        "two requests ran together under a one-problem budget"
    assert st["held_bytes"] <= budget
    # FIFO admission
    adm = [s[3]["admitted"] for s in served]
    assert adm == sorted(adm)


def test_cancel_queued_request():
    from paper_1607_00315_amd import sic
    probs = _mix(count=3, seed=25, n_lo=900, n_hi=1100)
    announce("one slot, three requests, cancel the last before admission")
    with sic.Server(slots=1) as srv:
        tickets = [srv.submit(p) for p in probs]
        assert srv.cancel(tickets[2])
        r2 = srv.wait(tickets[2], timeout=60.0)
        r0 = srv.wait(tickets[0], timeout=300.0)
        r1 = srv.wait(tickets[1], timeout=300.0)
    assert r2[0] == sic.SIC_ECANCELED and r2[1][0] is None
    assert r0[0] == 0 and r1[0] == 0


def test_lambda_path_request_equals_batch():
    from paper_1607_00315_amd import sic
    X, P, spec = workload("random_n600_m300")
    path = [0.4, 0.3, 0.2]
    announce("lambda path random_n600_m300 as one served request and as a batch")
    req = dict(X=X, lambda_path=path, tol=TOL)
    with sic.Server(slots=2, block=spec["block"]) as srv:
        other = srv.submit(_mix(count=1, seed=26, n_lo=800, n_hi=800)[0])
        t = srv.submit(req)
        code, results, infos, _ = srv.wait(t, timeout=300.0)
        assert srv.wait(other, timeout=300.0)[0] == 0
    with sic.Context(block=spec["block"]) as c:
        bcode, bres = c.solve_batch([req])
    assert code == bcode == 0
    assert len(results) == len(bres) == len(path)
    for (A, info), a in zip(bres, results):
        _same(a, A, X.shape[1])
        assert info["status"] == 0
