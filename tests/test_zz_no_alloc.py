"""The no-allocation inverse-column solve against the allocating one.

sic_step_inverse_columns_noalloc runs the block conjugate gradients of
Section 6.1 with every buffer in a static per-device array. Its results must
equal sic_step_inverse_columns' (same kernels, same launch shapes, so the
same arithmetic) on two calls in a row, the second on a smaller problem, so
that whatever the first call left in the array cannot leak into the second.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from synth import workload
from tests.helpers import announce

pytestmark = pytest.mark.gpu


def _csr(P):
    M = sp.csr_matrix(P)
    M.sort_indices()
    return M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.float64)


def _case(sic, torch, ctx, name, cols, tol):
    X, P, spec = workload(name)
    n = X.shape[1]
    rp, col, val = _csr(P)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    prob = sic.Prob(ctx, X, spec["lam"])
    try:
        prob.set_A(rp, col, val)
        W_ref, it_ref, res_ref = prob.inverse_columns(cols, tol=tol, max_iter=2000)
    finally:
        prob.close()
    dev = torch.device("cuda:0")
    d_rp, d_col, d_val = (torch.from_numpy(a).to(dev) for a in (rp, col, val))
    d_cols = torch.from_numpy(cols).to(dev)
    W = torch.full((n, cols.size), float("nan"), dtype=torch.float64, device=dev)
    assert sic.inverse_columns_noalloc_limit(n, col.size, cols.size) > 0
    it, res = sic.inverse_columns_noalloc(d_rp, d_col, d_val, d_cols, W, tol=tol, max_iter=2000)
    torch.cuda.synchronize()
    W = W.cpu().numpy()
    assert it == it_ref and res == res_ref, (it, it_ref, res, res_ref)
    assert res <= tol
    assert np.array_equal(W, W_ref), float(np.max(np.abs(W - W_ref)))
    # and the columns solve A W = E_cols
    E = np.zeros_like(W)
    E[cols, np.arange(cols.size)] = 1.0
    assert np.max(np.abs(sp.csr_matrix((val, col, rp), shape=(n, n)) @ W - E)) <= 1e-8


def test_noalloc_inverse_columns_equal_the_allocating_ones():
    import torch
    from paper_1607_00315_amd import sic
    rng = np.random.default_rng(11)
    with sic.Context() as ctx:
        announce("noalloc CG: grid_n2500_m1500, 200 columns (4 tiles, ragged) vs sic_step_inverse_columns")
        _case(sic, torch, ctx, "grid_n2500_m1500", rng.choice(2500, 200, replace=False), 1e-12)
        announce("noalloc CG: second call, smaller: grid_n400_m300, 70 columns")
        _case(sic, torch, ctx, "grid_n400_m300", rng.choice(400, 70, replace=False), 1e-12)


def test_noalloc_refuses_too_large_a_solve():
    import torch
    from paper_1607_00315_amd import sic
    announce("noalloc CG: a solve beyond the scratch array is refused with SIC_ETOOBIG")
    n, k = 200_000, 256
    assert sic.inverse_columns_noalloc_limit(n, n, k) == 0
    dev = torch.device("cuda:0")
    rp = torch.arange(n + 1, dtype=torch.int64, device=dev)
    col = torch.arange(n, dtype=torch.int32, device=dev)
    val = torch.ones(n, dtype=torch.float64, device=dev)
    cols = torch.arange(k, dtype=torch.int32, device=dev)
    W = torch.empty((n, k), dtype=torch.float64, device=dev)
    with pytest.raises(sic.SicError) as e:
        sic.inverse_columns_noalloc(rp, col, val, cols, W)
    assert e.value.code == sic.SIC_ETOOBIG
