"""Drawing the request stream's Gaussian samples on the GPU.

The serving workload needs hundreds of sample matrices of up to 4000 x 8000;
drawing them on the host takes tens of seconds each. This module draws from
the same law as :func:`synth.generators.sample_gaussian` (same precision
matrix, same split P = G G^T, same Chebyshev solve of P y = G xi on the
Jacobi-scaled system), with torch on a device and the normal draws from a
seeded torch generator, so the bytes differ from the host sampler's but the
distribution does not. Like the rest of ``synth`` it holds none of the
estimator's arithmetic.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .generators import _precision, _split_gram_factor


def _to_torch_csr(M: sp.csr_matrix, device):
    import torch
    M = sp.csr_matrix(M, dtype=np.float64)
    return torch.sparse_csr_tensor(torch.from_numpy(M.indptr.astype(np.int64)),
                                   torch.from_numpy(M.indices.astype(np.int64)),
                                   torch.from_numpy(M.data), size=M.shape,
                                   dtype=torch.float64).to(device)


def sample_gaussian_device(P: sp.csr_matrix, m: int, seed: int, device="cuda:0",
                           rtol: float = 1e-14, max_iter: int = 5000):
    """m samples of N(0, P^{-1}) as an m x n float64 tensor on ``device``."""
    import torch
    P = sp.csr_matrix(P, dtype=np.float64)
    n = P.shape[0]
    G = _split_gram_factor(P)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    xi = torch.randn((G.shape[1], m), generator=gen, dtype=torch.float64, device=device)
    Z = _to_torch_csr(G, device) @ xi
    del xi
    dg = P.diagonal()
    off = np.asarray(abs(P).sum(axis=1)).ravel() - np.abs(dg)
    rho = float(np.max(off / dg))
    if not rho < 1.0:
        raise ValueError("Jacobi-scaled spectrum bound needs strict dominance")
    s = 1.0 / np.sqrt(dg)
    Ps = _to_torch_csr((sp.diags(s) @ P @ sp.diags(s)).tocsr(), device)
    st = torch.from_numpy(s).to(device)[:, None]
    B = Z * st
    del Z
    lo, hi = 1.0 - rho, 1.0 + rho
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    x = torch.zeros_like(B)
    r = B.clone()
    bnorm = torch.linalg.vector_norm(B, dim=0).clamp_min(1e-300)
    del B
    rho_k = 1.0 / sigma
    d = r / theta
    for it in range(max_iter):
        x += d
        r -= Ps @ d
        if it % 8 == 7:
            rel = float((torch.linalg.vector_norm(r, dim=0) / bnorm).max())
            if rel <= rtol:
                break
        rho_next = 1.0 / (2.0 * sigma - rho_k)
        d *= rho_next * rho_k
        d += (2.0 * rho_next / delta) * r
        rho_k = rho_next
    else:
        raise RuntimeError("Chebyshev sampling solve did not converge")
    return (x * st).T.contiguous()


def request_samples_device(req: dict, device="cuda:0"):
    """The samples of one request of :func:`synth.generators.request_stream`,
    drawn on the device (the precision matrix is the host sampler's)."""
    rng = np.random.default_rng(req["seed"])
    P = _precision(req["kind"], req["n"], rng, 3)
    return sample_gaussian_device(P, req["m"], int(rng.integers(0, 2**62)), device), P
