"""Per-step parity of the HIP path against the CPU oracle, through the C-ABI.

Integer outputs (free sets, neighbourhoods, coordinates, hierarchy) must match
bit for bit; floating-point outputs within the tolerances stated per test,
derived from the arithmetic (float64 throughout):
  * S_J: a length-m dot product per entry, |error| <= m * eps * max|x|^2;
    checked at 1e-12 relative to max|S|.
  * W_J: CG to relative residual 1e-12 on matrices with condition < 100;
    checked at 1e-9 absolute.
  * CD / line search on identical inputs: only the summation order differs
    (the GPU updates the Hessian term incrementally); 1e-10 after a fixed
    number of sweeps.
"""

import numpy as np
import pytest

from oracle import core, steps
from oracle.cd import cd_sweeps
from oracle.quic_plain import linesearch_dense, objective_change
from synth import workload
from tests.helpers import announce, csr_to_dense, dense_to_csr, check_csr_valid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1607_00315_amd import sic
    import torch
    assert torch.cuda.is_available()
    c = sic.Context(block=128)
    yield c
    c.close()


@pytest.fixture(scope="module")
def rnd600():
    X, P, spec = workload("random_n600_m300")
    return X, P, spec, core.covariance(X)


def _prob(ctx, X, lam):
    from paper_1607_00315_amd import sic
    return sic.Prob(ctx, X, lam)


# ---------------------------------------------------------------- (a) S_J

@pytest.mark.parametrize("j0,b", [(0, 128), (512, 88), (300, 1), (100, 64)])
def test_cov_block(ctx, rnd600, j0, b):
    X, P, spec, S = rnd600
    announce(f"cov_block random_n600 j0={j0} b={b}")
    pr = _prob(ctx, X, spec["lam"])
    got = pr.cov_block(j0, b)
    ref = steps.cov_block(X, j0, j0 + b)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_cov_block_many_samples():
    from paper_1607_00315_amd import sic
    X, P, spec = workload("grid_n2500_m1500")
    announce("cov_block grid_n2500_m1500 j0=2304 b=196")
    with sic.Context(block=256) as c:
        pr = sic.Prob(c, X, spec["lam"])
        got = pr.cov_block(2304, 196)
        pr.close()
    ref = steps.cov_block(X, 2304, 2500)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def _narrow(X, dtype):
    """X rounded to float or to bfloat16 (nearest even), back in float64."""
    x32 = np.asarray(X, dtype=np.float32)
    if dtype == "f32":
        return x32.astype(np.float64)
    u = x32.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("name,j0,b", [("random_n600_m300", 512, 88),
                                       ("grid_n2500_m1500", 2304, 196)])
def test_cov_block_low(dtype, name, j0, b):
    """Reduced-precision S_J against the float64 product of the same narrowed
    samples, within the float accumulation bound gamma_(m+2) (|X|^T |X|)/m."""
    from paper_1607_00315_amd import sic
    X, P, spec = workload(name)
    m = X.shape[0]
    announce(f"cov_block_low {name} {dtype} j0={j0} b={b}")
    with sic.Context(block=256) as c:
        pr = sic.Prob(c, X, spec["lam"])
        got = pr.cov_block_low(j0, b, sic.SIC_X_F32 if dtype == "f32" else sic.SIC_X_BF16)
        pr.close()
    Xn = _narrow(X, dtype)
    ref = Xn.T @ Xn[:, j0:j0 + b] / m
    u = 2.0 ** -24
    gam = (m + 2) * u / (1 - (m + 2) * u)
    bound = gam * (np.abs(Xn).T @ np.abs(Xn[:, j0:j0 + b])) / m
    assert np.all(np.abs(got - ref) <= bound + 1e-300)
    # and the narrowing itself is what separates it from float64 S
    full = steps.cov_block(X, j0, j0 + b)
    rel = np.max(np.abs(got - full)) / np.max(np.abs(full))
    assert rel < (2e-6 if dtype == "f32" else 2e-2)


def test_cov_pairs(ctx, rnd600):
    X, P, spec, S = rnd600
    announce("cov_pairs random_n600")
    rng = np.random.default_rng(0)
    r = rng.integers(0, 600, 777).astype(np.int32)
    c = rng.integers(0, 600, 777).astype(np.int32)
    pr = _prob(ctx, X, spec["lam"])
    got = pr.cov_pairs(r, c)
    ref = np.einsum("ij,ij->j", X[:, r], X[:, c]) / X.shape[0]
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(S))


# ---------------------------------------------------------------- (b) W_J

@pytest.mark.parametrize("k", [1, 70, 200])
def test_inverse_columns(ctx, rnd600, k):
    X, P, spec, S = rnd600
    announce(f"inverse_columns random_n600 k={k}")
    rng = np.random.default_rng(k)
    cols = np.sort(rng.choice(600, size=k, replace=False)).astype(np.int32)
    pr = _prob(ctx, X, spec["lam"])
    Ad = P.toarray()
    pr.set_A(*dense_to_csr(Ad))
    W, it, res = pr.inverse_columns(cols, tol=1e-12, max_iter=2000)
    ref = steps.inverse_columns(Ad, cols)
    assert res <= 1e-12 and it > 0
    assert np.max(np.abs(W - ref)) <= 1e-9


# ---------------------------------------------------------------- (d) CD, (e) line search

def _block_inputs(A, S, lam, j0, j1, candidates=None):
    W = core.inverse_pd(A)
    G_J = S[:, j0:j1] - W[:, j0:j1]
    free = steps.screen(G_J, A[:, j0:j1], lam, j0, j1, candidates)
    r, c = steps.coordinates(free, j0, j1)
    N = steps.neighborhood(free, j0, j1)
    Jp = steps.local_set(j0, j1, N)
    loc = {int(g): k for k, g in enumerate(Jp)}
    cp = np.array([loc[int(x)] for x in r], dtype=np.int32)
    b = j1 - j0
    cptr = np.zeros(b + 1, dtype=np.int64)
    np.add.at(cptr, (c - j0) + 1, 1)
    cptr = np.cumsum(cptr)
    wjj = W[np.ix_(Jp, Jp)]
    return dict(W=W, free=free, r=r, c=c, N=N, Jp=Jp, cp=cp, cptr=cptr, wjj=wjj,
                S=S[r, c], A=A[r, c], b=b)


def _mlbcd_iterate(X, lam, b, sweeps=1):
    from oracle import mlbcd
    S = core.covariance(X)
    A = np.eye(S.shape[0])
    for _ in range(sweeps):
        A, _, _, _, _ = mlbcd.relax(A, S, lam, b)
    return A, S


@pytest.fixture(scope="module")
def ctx_u():
    """Context whose CD always takes the U = Delta W form."""
    from paper_1607_00315_amd import sic
    c = sic.Context(block=128, cd_hessian_max=-1)
    yield c
    c.close()


@pytest.mark.parametrize("form", ["hessian", "u"])
@pytest.mark.parametrize("start", ["identity", "iterate"])
def test_cd_step_matches_oracle(ctx, ctx_u, rnd600, start, form):
    """Both CD forms against the plain C loop; the identity start has 2630
    coordinates (42 chunks of 64, the last one ragged)."""
    from paper_1607_00315_amd import sic
    X, P, spec, S = rnd600
    lam = spec["lam"]
    A = np.eye(600) if start == "identity" else _mlbcd_iterate(X, lam, 128)[0]
    j0, j1 = 128, 256
    d = _block_inputs(A, S, lam, j0, j1)
    ctx = ctx if form == "hessian" else ctx_u
    announce(f"step_cd random_n600 start={start} form={form} coords={d['r'].size} |N|={d['N'].size}")
    # fixed number of sweeps: identical work on both sides
    got, st = sic.step_cd(ctx, d["wjj"], d["b"], d["cptr"], d["cp"], d["S"], d["A"], lam,
                          max_sweeps=6, tol=0.0)
    ref, sw, _ = cd_sweeps(d["wjj"], d["cp"], d["c"] - j0, d["S"], d["A"], lam, 6, 0.0)
    assert int(st[0]) == sw == 6
    assert np.max(np.abs(got - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
    # default stopping rule: same answer within the inner tolerance
    got2, st2 = sic.step_cd(ctx, d["wjj"], d["b"], d["cptr"], d["cp"], d["S"], d["A"], lam)
    ref2, sw2, _ = steps.cd_block(d["W"], d["r"], d["c"], d["S"], d["A"], lam, j0, j1, d["N"])
    assert abs(int(st2[0]) - sw2) <= 1
    assert np.max(np.abs(got2 - ref2)) <= 1e-3 * max(1e-12, np.max(np.abs(ref2)))


@pytest.mark.parametrize("j1,lam_scale,chunks", [(160, 1.0, 12), (176, 1.0, 18), (130, 1.0, 3),
                                                 (129, 1.0, 2), (129, 1.5, 1), (129, 3.0, 1)])
def test_cd_multi_step_matches_oracle(ctx, rnd600, j1, lam_scale, chunks):
    """The multi-workgroup explicit-Hessian sweep (the kernel of the benchmark's
    blocks): 718 coordinates (12 chunks, the last ragged, one helper workgroup
    each) and 1137 (18 chunks, two helpers owning two chunks), and the cases
    with fewer chunks than the snapshot lag of three intervals (3, 2, 1 chunks,
    down to a single coordinate); six fixed sweeps against the plain C loop,
    then the default stopping rule against the oracle."""
    from paper_1607_00315_amd import sic
    X, P, spec, S = rnd600
    lam = spec["lam"] * lam_scale
    j0 = 128
    d = _block_inputs(np.eye(600), S, lam, j0, j1)
    assert (d["r"].size + 63) // 64 == chunks
    announce(f"step_cd (multi-workgroup) random_n600 block [{j0},{j1}) lam={lam} "
             f"coords={d['r'].size}")
    got, st = sic.step_cd(ctx, d["wjj"], d["b"], d["cptr"], d["cp"], d["S"], d["A"], lam,
                          max_sweeps=6, tol=0.0)
    ref, sw, _ = cd_sweeps(d["wjj"], d["cp"], d["c"] - j0, d["S"], d["A"], lam, 6, 0.0)
    # with tol = 0 a sweep stops the loop only when every step is exactly zero:
    # either side can reach such a fixed point early on a small block (more
    # sweeps would keep it); the summation orders differ, so one may stop while
    # the other keeps taking steps of rounding size
    assert 1 <= sw <= 6 and 1 <= int(st[0]) <= 6
    if chunks > 3:
        assert int(st[0]) == sw == 6
    assert np.max(np.abs(got - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
    got2, st2 = sic.step_cd(ctx, d["wjj"], d["b"], d["cptr"], d["cp"], d["S"], d["A"], lam)
    ref2, sw2, _ = steps.cd_block(d["W"], d["r"], d["c"], d["S"], d["A"], lam, j0, j1, d["N"])
    assert abs(int(st2[0]) - sw2) <= 1
    assert np.max(np.abs(got2 - ref2)) <= 1e-3 * max(1e-12, np.max(np.abs(ref2)))


@pytest.fixture(scope="module")
def ctx_pcd():
    """Context whose blocks all take the PCD-CG direction."""
    from paper_1607_00315_amd import sic
    c = sic.Context(block=128, pcd_min_coords=1)
    yield c
    c.close()


@pytest.mark.parametrize("start", ["identity", "iterate"])
def test_pcd_step_matches_oracle(ctx_pcd, rnd600, start):
    """PCD-CG against the oracle's PCD-CG: the same iterations (10 line
    searches, no stop test), the default stopping rule, and run to convergence
    against the cyclic-CD minimiser of the same block model."""
    from oracle import pcd
    from paper_1607_00315_amd import sic
    X, P, spec, S = rnd600
    lam = spec["lam"]
    A = np.eye(600) if start == "identity" else _mlbcd_iterate(X, lam, 128)[0]
    j0, j1 = 128, 256
    d = _block_inputs(A, S, lam, j0, j1)
    ci = d["c"] - j0
    announce(f"step_cd (PCD-CG) random_n600 start={start} coords={d['r'].size} |N|={d['N'].size}")
    got, st = sic.step_cd(ctx_pcd, d["wjj"], d["b"], d["cptr"], d["cp"], d["S"], d["A"], lam,
                          max_sweeps=1, tol=0.0)
    ref, its, _ = pcd.pcd_cg(d["wjj"], d["cp"], ci, d["S"], d["A"], lam, max_iter=10, tol=0.0)
    if start == "iterate":
        assert int(st[0]) == its
    # at the identity start W = I makes the model separable: the first PCD step
    # is its exact minimiser and the later line searches act on rounding noise,
    # so the two sides may stop after different counts at the same answer
    scale = max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(got - ref)) <= 1e-9 * scale
    assert np.array_equal(got == -d["A"], ref == -d["A"])      # exact zeros agree
    got2, st2 = sic.step_cd(ctx_pcd, d["wjj"], d["b"], d["cptr"], d["cp"], d["S"], d["A"], lam)
    ref2, its2, _ = pcd.pcd_cg(d["wjj"], d["cp"], ci, d["S"], d["A"], lam)
    assert abs(int(st2[0]) - its2) <= 1
    assert np.max(np.abs(got2 - ref2)) <= 1e-3 * max(1e-12, np.max(np.abs(ref2)))
    got3, st3 = sic.step_cd(ctx_pcd, d["wjj"], d["b"], d["cptr"], d["cp"], d["S"], d["A"], lam,
                            max_sweeps=100, tol=1e-12)
    ref3, _, _ = cd_sweeps(d["wjj"], d["cp"], ci, d["S"], d["A"], lam, 1000, 1e-14)
    assert np.max(np.abs(got3 - ref3)) <= 1e-7 * max(1.0, np.max(np.abs(ref3)))
    assert np.array_equal(got3 + d["A"] == 0, ref3 + d["A"] == 0)


@pytest.mark.parametrize("start", ["identity", "iterate"])
def test_linesearch_step_matches_oracle(ctx, rnd600, start):
    from paper_1607_00315_amd import sic
    X, P, spec, S = rnd600
    lam = spec["lam"]
    A = np.eye(600) if start == "identity" else _mlbcd_iterate(X, lam, 128)[0]
    j0, j1 = 256, 384
    d = _block_inputs(A, S, lam, j0, j1)
    Dv, _, _ = steps.cd_block(d["W"], d["r"], d["c"], d["S"], d["A"], lam, j0, j1, d["N"])
    announce(f"step_linesearch random_n600 start={start} coords={d['r'].size}")
    D = steps.delta_matrix(600, d["r"], d["c"], Dv)
    alpha, dF, trials, ld = sic.step_linesearch(ctx, d["wjj"], d["b"], d["cptr"], d["cp"],
                                                d["S"], d["A"], Dv, lam, n_alpha=6)
    L = np.linalg.cholesky(A)
    ld0 = 2 * np.sum(np.log(np.diag(L)))
    for i in range(6):
        a = 0.5 ** i
        ref = core.logdet_pd(A + a * D)
        if ref is None:
            assert np.isnan(ld[i])
        else:
            assert ld[i] == pytest.approx(ref - ld0, abs=1e-10)
    a_ref, dF_ref, tr_ref = linesearch_dense(A, D, S, lam)
    assert alpha == a_ref
    assert dF == pytest.approx(dF_ref, rel=1e-9, abs=1e-13)
    assert dF < 0


def test_linesearch_rejects_non_pd_full_step(ctx):
    """A direction whose full step leaves the PD cone: alpha < 1 and the
    non-PD trial is skipped (Section 6.1.2, eq. (Schurs_PDness))."""
    from paper_1607_00315_amd import sic
    n, b = 6, 3
    A = np.eye(n)
    S = np.eye(n) * 2.0
    # coordinates: the diagonal of the block, Delta_00 = -1.5 makes alpha=1 non-PD
    cptr = np.array([0, 1, 2, 3], dtype=np.int64)
    cp = np.array([0, 1, 2], dtype=np.int32)
    Dv = np.array([-1.5, 0.0, 0.0])
    wjj = np.eye(b)
    alpha, dF, trials, ld = sic.step_linesearch(ctx, wjj, b, cptr, cp, S[[0, 1, 2], [0, 1, 2]],
                                                A[[0, 1, 2], [0, 1, 2]], Dv, 0.0, n_alpha=3)
    D = np.zeros((n, n)); D[0, 0] = -1.5
    a_ref, dF_ref, _ = linesearch_dense(A, D, S, 0.0)
    assert np.isnan(ld[0])
    assert alpha == a_ref
    assert dF == pytest.approx(dF_ref, rel=1e-12)


# ---------------------------------------------------------------- full block update

def _compare_block(pr, res, ref, j0, b, A_dense):
    out = pr.last_block(res, b)
    # free set per column, bit-exact
    for ci in range(b):
        rows = out["rows"][out["colptr"][ci]:out["colptr"][ci + 1]]
        assert np.array_equal(rows, ref["free"][ci]), f"free set differs in column {j0 + ci}"
    assert np.array_equal(out["nbrs"], ref["N"])
    assert np.array_equal(out["coord_rows"], ref["r"])
    assert np.array_equal(out["coord_cols"], ref["c"])
    assert np.max(np.abs(out["delta"] - ref["D_vals"])) <= 1e-6 * max(1.0, np.max(np.abs(ref["D_vals"])))
    assert res["alpha"] == ref["alpha"]
    assert res["dF"] == pytest.approx(ref["dF"], rel=1e-6, abs=1e-12)


@pytest.mark.parametrize("start,j0,b", [("identity", 128, 128), ("iterate", 512, 88),
                                        ("iterate", 0, 128)])
def test_block_update_finest_level(ctx, rnd600, start, j0, b):
    X, P, spec, S = rnd600
    lam = spec["lam"]
    A = np.eye(600) if start == "identity" else _mlbcd_iterate(X, lam, 128)[0]
    announce(f"block finest random_n600 start={start} j0={j0} b={b}")
    pr = _prob(ctx, X, lam)
    pr.set_A(*dense_to_csr(A))
    res = pr.block(j0, b, level=0, tol_I=1e-12, tol_N=1e-12)
    ref = steps.block_update(A, S, j0, j0 + b, lam)
    _compare_block(pr, res, ref, j0, b, A)
    rp, col, val = pr.get_A()
    check_csr_valid(rp, col, val, 600)
    Anew = csr_to_dense(rp, col, val, 600)
    assert np.array_equal(Anew, Anew.T)
    assert np.array_equal(Anew != 0, ref["A_new"] != 0)
    assert np.max(np.abs(Anew - ref["A_new"])) <= 1e-6


def test_block_update_coarse_level(ctx, rnd600):
    X, P, spec, S = rnd600
    lam = spec["lam"]
    A, _ = _mlbcd_iterate(X, lam, 128)
    n = 600
    supp = core.support_pairs(A)
    # level set: the support plus a seeded selection of other pairs
    rng = np.random.default_rng(5)
    iu, ju = np.triu_indices(n, 1)
    extra = rng.choice(iu.size, size=3000, replace=False)
    keys = np.union1d(supp, iu[extra].astype(np.int64) * n + ju[extra])
    cand = steps.level_candidates(keys, keys.size, n)
    j0, b = 256, 128
    announce(f"block coarse random_n600 j0={j0} |C|={keys.size}")
    pr = _prob(ctx, X, lam)
    pr.set_A(*dense_to_csr(A))
    pr.set_level(keys)
    res = pr.block(j0, b, level=1, tol_I=1e-12, tol_N=1e-12)
    ref = steps.block_update(A, S, j0, j0 + b, lam, candidates=cand)
    _compare_block(pr, res, ref, j0, b, A)
    rp, col, val = pr.get_A()
    Anew = csr_to_dense(rp, col, val, n)
    assert np.array_equal(Anew, Anew.T)
    assert np.max(np.abs(Anew - ref["A_new"])) <= 1e-6
    # the update stays inside the level set
    assert np.all(np.isin(core.support_pairs(Anew), keys))
