"""Write the stored expected values of the named workloads (calls only the oracle).

For each workload: the oracle minimiser A* (dense proximal Newton to a KKT
max-norm of 1e-10), its objective F*, support keys and the oracle's own
per-iteration history (objective, KKT, seconds). Usage:

    python tests/golden/make_golden.py grid_n10000_m5000 [more names]
"""

from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import core, quic_plain  # noqa: E402
from synth import workload  # noqa: E402


def main(names):
    for name in names:
        X, P, spec = workload(name)
        lam = spec["lam"]
        S = core.covariance(X)
        t0 = time.perf_counter()
        A, info = quic_plain.solve(S, lam, tol=1e-10, verbose=True)
        secs = time.perf_counter() - t0
        keys = core.support_pairs(A)
        out = dict(
            workload=name, n=int(S.shape[0]), m=int(X.shape[0]), lam=lam,
            F_star=info["objective"], kkt_max=info["kkt_max"], kkt_l1=info["kkt_l1"],
            nnz=int(np.count_nonzero(A)), support_pairs=int(keys.size),
            support_sha256=hashlib.sha256(keys.tobytes()).hexdigest(),
            oracle_seconds=secs, oracle_threads=os.cpu_count(),
            history=[dict(iteration=h[0], F=h[1], kkt_max=h[2], nnz=h[3], seconds=h[4])
                     for h in info["history"]],
            source="oracle.quic_plain.solve(tol=1e-10) on synth.workload(name)",
        )
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        np.savez_compressed(os.path.join(HERE, f"{name}_support.npz"), keys=keys)
        print(f"[golden] {name}: F*={out['F_star']:.15e} kkt={out['kkt_max']:.2e} "
              f"nnz={out['nnz']} in {secs:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["chain_n200_m100"])
